// Device-side Ritz analysis of the Arnoldi Hessenberg matrix (one wavefront).
//
// Ritz pairs (mu_H, y) of H_p give the approximations (mu, V_p y) of the
// eigenpairs of M (Sec. 3.2.1, eq. "m-step Arnoldi" and the Ritz relation that
// follows it); each pair is judged by |beta e_p^T y| with ||y|| = 1 (Sec. 3.2.2,
// eq. "Krylov convergence").  The eigensolver is the shifted QR algorithm on the
// Hessenberg matrix in complex arithmetic (Francis 1961; Golub & Van Loan,
// "Matrix Computations", Sec. 7.5): Wilkinson shift from the trailing 2x2
// block, an exceptional shift every tenth iteration, deflation on negligible
// subdiagonal entries, Givens rotations accumulated into Z so that
// H = Z T Z^H with T upper triangular.  A real H (real operators) is treated as
// complex; its conjugate pairs come out to rounding.
//
// Wavefront design.  The whole solve runs in one 64-lane wavefront, so every
// wait is just the LDS latency of one wave.  T (p x p complex128, row-major)
// sits in LDS.  The deflation test of all subdiagonal entries is one ballot.
// Every lane evaluates the shift and the rotation of the current bulge position
// itself from broadcast LDS reads.  The similarity G T G^H of one rotation
// touches two rows and two columns whose only overlap is a 2x2 block, so the
// block, the rest of the rows and the rest of the columns are updated in a
// single phase: one wait per rotation.  For the Arnoldi stop test only the
// last row of Z (H = Z T Z^H) is tracked: with z_i the eigenvectors of T (back
// substitution, one eigenvector per lane, no synchronisation) and Z unitary,
// the residual of Ritz pair i is beta |(last row of Z) z_i| / ||z_i||.  The
// unit Ritz coordinates of the wanted pairs are then computed once, at the end
// of the run, by inverse iteration on H (k_ritz_coords).  The standalone entry
// point accumulates all of Z instead (rotations recorded per sweep and applied
// to Z off the critical path) and forms every eigenvector.
//
// Wanted set (stop rule documented with tsk_arnoldi): sort by |mu| descending
// (ties: larger arg mu first), accept converged values, skip an unconverged
// value that lies within its residual of a converged or an already accepted
// value, accept the rest; done when the first k accepted are converged.  With
// dup_rel > 0 (FP32 states) values closer than dup_rel |mu| to an accepted or
// converged one also count as copies of it (FP32 rounding splits a multiple
// eigenvalue into a cluster of about that width), and a pair counts as
// converged below max(tol, res_floor |mu|), the FP32 floor of the estimate.
#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

constexpr int kHT = 64;  // one wavefront
constexpr double kEps = 2.220446049250313e-16;

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

// Givens rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0], c real:
// c = |x| / rho, s = (x/|x|) conj(y) / rho, rho = sqrt(|x|^2 + |y|^2).  The
// rotation is on the critical path of the bulge chase, so it is built from one
// reciprocal square root: with f = (|x|^2 (|x|^2 + |y|^2))^(-1/2),
// c = |x|^2 f and s = x conj(y) f.  f starts from the hardware estimate and is
// refined by two Newton steps to full FP64 accuracy.  Arguments whose squares
// could leave the normal range take a scaled path.
__device__ inline double rsqrt_full(double v) {
    double y = __builtin_amdgcn_rsq(v);
    double h = 0.5 * v;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

__device__ inline void givens(double2 x, double2 y, double& c, double2& s) {
    const double nx = x.x * x.x + x.y * x.y, ny = y.x * y.x + y.y * y.y;
    if (ny == 0.0) { c = 1.0; s = cmk<double2>(0.0, 0.0); return; }
    if (nx == 0.0) {
        c = 0.0;
        const double f = 1.0 / sqrt(ny);
        s = cmk<double2>(y.x * f, -y.y * f);
        return;
    }
    const double q = nx * (nx + ny);
    if (q > 1e-280 && q < 1e280) {
        const double f = rsqrt_full(q);
        c = nx * f;
        s = cscale(cmulc(y, x), f);  // x conj(y) f
        return;
    }
    const double ax = sqrt(nx), rho = sqrt(nx + ny);
    const double f = 1.0 / (ax * rho);
    c = ax * f * ax;
    s = cscale(cmulc(y, x), f);
}

__device__ inline int highest_bit(unsigned long long m) { return 63 - __builtin_clzll(m); }

// z = eigenvector of upper-triangular T for eigenvalue index i (z[i] = 1,
// z[r > i] = 0), written to zc[0..i]; returns ||z||^2.
__device__ inline double tri_eigvec(const double2* T, int p, int i, double2* zc) {
    const double2 lam = T[i * p + i];
    double smin = kEps * cabs1(lam);
    if (smin < 1e-290) smin = 1e-290;
    zc[i] = cmk<double2>(1.0, 0.0);
    double nrm = 1.0;
    for (int c = i - 1; c >= 0; --c) {
        double2 acc = T[c * p + i];
        for (int r = c + 1; r < i; ++r) acc = cadd(acc, cmul(T[c * p + r], zc[r]));
        double2 den = csub(T[c * p + c], lam);
        if (cabs1(den) < smin) den = cmk<double2>(smin, 0.0);
        double2 z = cdiv(cmk<double2>(-acc.x, -acc.y), den);
        zc[c] = z;
        nrm += cabs2(z);
    }
    return nrm;
}

// FULLZ: accumulate all of Z (standalone use, every eigenvector formed);
// otherwise only the last row of Z is tracked (all the residuals need) and the
// wanted Ritz coordinates are computed afterwards by inverse iteration.
template <bool FULLZ>
__global__ __launch_bounds__(kHT) void k_hess_ritz(const KryDesc* __restrict__ Dv, int p, int k, double tol) {
    const KryDesc& dsc = Dv[blockIdx.x];
    if (!dsc.active) return;
    const double2* __restrict__ H = dsc.H;
    const int ldh = dsc.ldh;
    double2* __restrict__ Z = dsc.Z;
    double2* __restrict__ S = dsc.S;
    double2* __restrict__ mu = dsc.mu;
    double2* __restrict__ Y = dsc.Y;
    double* __restrict__ res = dsc.res;
    int* __restrict__ sel = dsc.sel;
    RitzResult* __restrict__ rr = dsc.rr;
    const double dup_rel = dsc.dup_rel;
    const double res_floor = dsc.res_floor;
    extern __shared__ double2 T[];  // p*p
    __shared__ double rc[kMaxKrylov];
    __shared__ double2 rs[kMaxKrylov];
    __shared__ double2 zl[kMaxKrylov];  // last row of Z
    __shared__ int order[kMaxKrylov];
    __shared__ int dupc[kMaxKrylov];
    __shared__ double znrm[kMaxKrylov];
    __shared__ double ctol[kMaxKrylov];  // per Ritz value convergence threshold
    const int lane = threadIdx.x;

    // beta_p: the Arnoldi path reads it from H's subdiagonal H[p][p-1], which
    // later (speculative) steps never modify; the standalone path from scal[2].
    const double beta = FULLZ ? dsc.scal[2] : H[p + (size_t)ldh * (p - 1)].x;
    bool bad = !isfinite(beta);
    for (int e = lane; e < p * p; e += kHT) {
        int r = e / p, c = e % p;
        const double2 v = (r <= c + 1) ? H[r + (size_t)ldh * c] : cmk<double2>(0.0, 0.0);
        bad = bad || !isfinite(v.x) || !isfinite(v.y);
        T[e] = v;
    }
    if (__ballot(bad)) {  // non-finite input: no QR (it could not deflate), report and stop
        if (lane == 0 && rr) {
            rr->nonfinite = 1;
            rr->done = 0;
            rr->nsel = 0;
            rr->nconv = 0;
            rr->eig_fail = FULLZ ? 1 : 0;
            rr->iters = 0;
        }
        return;
    }
    for (int c = lane; c < p; c += kHT) zl[c] = cmk<double2>(c == p - 1 ? 1.0 : 0.0, 0.0);
    if constexpr (FULLZ) {
        for (int r = lane; r < p; r += kHT)
            for (int c = 0; c < p; ++c) Z[c * p + r] = cmk<double2>(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    // ---- shifted QR iteration -------------------------------------------------------
    int ihi = p - 1, its = 0, total = 0, failed = 0;
    const int itmax = 30 * (p > 10 ? p : 10);
    while (ihi > 0) {
        // deflation: largest l <= ihi with a negligible T[l][l-1] (else 0)
        bool s0 = false, s1 = false;
        {
            int i = lane + 1;
            if (i <= ihi) {
                double tst = cabs1(T[(i - 1) * p + (i - 1)]) + cabs1(T[i * p + i]);
                if (tst == 0.0) tst = 1.0;
                s0 = cabs1(T[i * p + (i - 1)]) <= kEps * tst;
            }
            i = lane + 65;
            if (i <= ihi) {
                double tst = cabs1(T[(i - 1) * p + (i - 1)]) + cabs1(T[i * p + i]);
                if (tst == 0.0) tst = 1.0;
                s1 = cabs1(T[i * p + (i - 1)]) <= kEps * tst;
            }
        }
        unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
        int l = m1 ? highest_bit(m1) + 65 : (m0 ? highest_bit(m0) + 1 : 0);
        __syncthreads();
        if (l > 0 && lane == 0) T[l * p + (l - 1)] = cmk<double2>(0.0, 0.0);
        __syncthreads();
        if (l == ihi) {
            --ihi;
            its = 0;
            continue;
        }
        if (++total > itmax) { failed = 1; break; }
        ++its;
        // shift (every lane computes it)
        double2 sft;
        {
            double2 a = T[(ihi - 1) * p + (ihi - 1)], b = T[(ihi - 1) * p + ihi];
            double2 c2 = T[ihi * p + (ihi - 1)], d = T[ihi * p + ihi];
            if (its % 10 == 0) {
                double ex = 0.75 * fabs(c2.x) + fabs(d.x);
                sft = cmk<double2>(d.x + ex, d.y);
            } else {
                double2 half = cscale(csub(a, d), 0.5);
                double2 disc = csqrt(cadd(cmul(half, half), cmul(b, c2)));
                double2 mid = cscale(cadd(a, d), 0.5);
                double2 l1 = cadd(mid, disc), l2 = csub(mid, disc);
                sft = (cabs(csub(l1, d)) <= cabs(csub(l2, d))) ? l1 : l2;
            }
        }
        // Bulge chase kk = l .. ihi-1.  The similarity G T G^H touches rows
        // {kk, kk+1} (left factor) and columns {kk, kk+1} (right factor); apart
        // from their 2x2 intersection the two sets are disjoint, so one phase
        // (one wait) per rotation updates: the 2x2 block, the rest of the two
        // rows (columns kk-1 and kk+2..p-1) and the rest of the two columns
        // (rows 0..kk-1 and kk+2).
        for (int kk = l; kk < ihi; ++kk) {
            double2 x, y;
            if (kk == l) {
                x = csub(T[l * p + l], sft);
                y = T[(l + 1) * p + l];
            } else {
                x = T[kk * p + (kk - 1)];
                y = T[(kk + 1) * p + (kk - 1)];
            }
            double c;
            double2 s;
            givens(x, y, c, s);
            const double2 sc = cconj(s);
            const int nrow_only = (p - (kk + 2) > 0 ? p - (kk + 2) : 0);  // columns kk+2..p-1
            const int ncol_only = kk + (kk + 2 <= ihi ? 1 : 0);            // rows 0..kk-1, kk+2
            const int items = nrow_only + ncol_only;
            // 2x2 block G B G^H, the annihilated bulge column and the last row of
            // Z: every lane computes them (uniform control flow), lane 0 stores.
            {
                double2 a = T[kk * p + kk], b = T[kk * p + kk + 1];
                double2 d = T[(kk + 1) * p + kk], e = T[(kk + 1) * p + kk + 1];
                double2 za = zl[kk], zb = zl[kk + 1];
                double2 a1 = cadd(cscale(a, c), cmul(s, d)), b1 = cadd(cscale(b, c), cmul(s, e));
                double2 d1 = csub(cscale(d, c), cmul(sc, a)), e1 = csub(cscale(e, c), cmul(sc, b));
                a = cadd(cscale(a1, c), cmul(sc, b1));
                b = csub(cscale(b1, c), cmul(s, a1));
                d = cadd(cscale(d1, c), cmul(sc, e1));
                e = csub(cscale(e1, c), cmul(s, d1));
                double2 xn = cadd(cscale(x, c), cmul(s, y));
                double2 za1 = cadd(cscale(za, c), cmul(sc, zb)), zb1 = csub(cscale(zb, c), cmul(s, za));
                if (lane == 0) {
                    T[kk * p + kk] = a;
                    T[kk * p + kk + 1] = b;
                    T[(kk + 1) * p + kk] = d;
                    T[(kk + 1) * p + kk + 1] = e;
                    if (kk > l) {
                        T[kk * p + (kk - 1)] = xn;
                        T[(kk + 1) * p + (kk - 1)] = cmk<double2>(0.0, 0.0);
                    }
                    zl[kk] = za1;
                    zl[kk + 1] = zb1;
                    rc[kk - l] = c;
                    rs[kk - l] = s;
                }
            }
            // one entry pair per lane: rows {kk, kk+1} at a column outside the
            // block (left factor), or columns {kk, kk+1} at a row outside it
            // (right factor); both are (u, v) -> (c u + s1 v, c v - s2 u)
            for (int t = lane; t < items; t += kHT) {
                const bool rowop = t < nrow_only;
                int ia, ib;
                if (rowop) {
                    const int col = kk + 2 + t;
                    ia = kk * p + col;
                    ib = (kk + 1) * p + col;
                } else {
                    const int q = t - nrow_only;
                    const int row = q < kk ? q : kk + 2;
                    ia = row * p + kk;
                    ib = row * p + kk + 1;
                }
                const double2 s1 = rowop ? s : sc, s2 = rowop ? sc : s;
                const double2 u = T[ia], v = T[ib];
                T[ia] = cadd(cscale(u, c), cmul(s1, v));
                T[ib] = csub(cscale(v, c), cmul(s2, u));
            }
            __syncthreads();
        }
        if constexpr (FULLZ) {
            // Z <- Z G^H for the sweep's rotations, one row of Z per lane
            for (int row = lane; row < p; row += kHT) {
                double2 carry = Z[l * p + row];
                for (int kk = l; kk < ihi; ++kk) {
                    const double c = rc[kk - l];
                    const double2 s = rs[kk - l];
                    double2 b = Z[(kk + 1) * p + row];
                    Z[kk * p + row] = cadd(cscale(carry, c), cmul(cconj(s), b));
                    carry = csub(cscale(b, c), cmul(s, carry));
                }
                Z[ihi * p + row] = carry;
            }
            __syncthreads();
        }
    }

    // ---- Ritz values and residuals ---------------------------------------------------------
    for (int i = lane; i < p; i += kHT) {
        mu[i] = T[i * p + i];
        double2* zc = S + (size_t)i * p;
        double n2 = tri_eigvec(T, p, i, zc);
        double2 last = cmk<double2>(0.0, 0.0);
        for (int c = 0; c <= i; ++c) last = cadd(last, cmul(zl[c], zc[c]));
        double nz = sqrt(n2);
        znrm[i] = nz;
        res[i] = fabs(beta) * cabs(last) / nz;
    }
    __syncthreads();

    if constexpr (FULLZ) {
        // every eigenvector: Y[:, i] = Z z_i / ||z_i||
        for (int i = 0; i < p; ++i) {
            const double2* zc = S + (size_t)i * p;
            const double inv = 1.0 / znrm[i];
            for (int r = lane; r < p; r += kHT) {
                double2 acc = cmk<double2>(0.0, 0.0);
                for (int c = 0; c <= i; ++c) acc = cadd(acc, cmul(Z[c * p + r], zc[c]));
                Y[(size_t)i * p + r] = cscale(acc, inv);
            }
        }
        if (lane == 0 && rr) { rr->eig_fail = failed; rr->iters = total; }
        return;
    } else {
        // ---- wanted set ------------------------------------------------------------------------
        // converged: res <= max(tol, res_floor |mu|)
        for (int i = lane; i < p; i += kHT) ctol[i] = fmax(tol, res_floor * cabs(mu[i]));
        __syncthreads();
        for (int i = lane; i < p; i += kHT) {
            double mi = cabs(mu[i]), ai = atan2(mu[i].y, mu[i].x);
            int rank = 0;
            for (int j = 0; j < p; ++j) {
                if (j == i) continue;
                double mj = cabs(mu[j]), aj = atan2(mu[j].y, mu[j].x);
                bool before = (mj > mi) || (mj == mi && (aj > ai || (aj == ai && j < i)));
                rank += before ? 1 : 0;
            }
            order[rank] = i;
            int d = 0;
            if (!(res[i] <= ctol[i])) {
                const double rad = fmax(res[i], dup_rel * cabs(mu[i]));
                for (int j = 0; j < p; ++j)
                    if (j != i && res[j] <= ctol[j] && cabs(csub(mu[i], mu[j])) <= rad) d = 1;
            }
            dupc[i] = d;
        }
        __syncthreads();
        if (lane == 0) {
            int nsel = 0, nconv = 0;
            for (int t = 0; t < p && nsel < k; ++t) {
                int i = order[t];
                bool conv = res[i] <= ctol[i];
                bool take;
                if (conv) {
                    // a converged copy of an accepted value (only with dup_rel > 0)
                    take = true;
                    const double rad = dup_rel * cabs(mu[i]);
                    for (int a = 0; a < nsel && take; ++a)
                        if (cabs(csub(mu[i], mu[sel[a]])) < rad) take = false;
                } else {
                    take = !dupc[i];
                    const double rad = fmax(res[i], dup_rel * cabs(mu[i]));
                    for (int a = 0; a < nsel && take; ++a)
                        if (cabs(csub(mu[i], mu[sel[a]])) <= rad) take = false;
                }
                if (take) {
                    sel[nsel++] = i;
                    nconv += conv ? 1 : 0;
                }
            }
            rr->nsel = nsel;
            rr->nconv = nconv;
            rr->done = (nsel >= k && nconv == nsel) ? 1 : 0;
            rr->eig_fail = failed;
            rr->iters = total;
        }
    }
}

// Unit Ritz coordinates of the wanted pairs by inverse iteration on H_p (one
// wavefront per pair): solve (H - mu I) y = b with the Hessenberg LU (partial
// pivoting between the two candidate rows of each column), twice, starting from
// b = (1, ..., 1); normalise to ||y|| = 1.  Y[s*p + r].
__global__ __launch_bounds__(kHT) void k_ritz_coords(const KryDesc* __restrict__ Dv) {
    const KryDesc& dsc = Dv[blockIdx.y];
    const int sidx = blockIdx.x;
    if (!dsc.ritz || sidx >= dsc.rr->nsel) return;
    const int p = dsc.steps;
    const double2* __restrict__ H = dsc.H;
    const int ldh = dsc.ldh;
    double2* __restrict__ Y = dsc.Y;
    extern __shared__ double2 A[];  // p*p, row-major
    __shared__ double2 b[kMaxKrylov];
    __shared__ int piv[kMaxKrylov];
    __shared__ double2 lmul[kMaxKrylov];
    __shared__ double red[kHT];
    const int lane = threadIdx.x;
    const double2 m = dsc.mu[dsc.sel[sidx]];
    double hn = 0.0;
    for (int e = lane; e < p * p; e += kHT) {
        int r = e / p, c = e % p;
        double2 v = (r <= c + 1) ? H[r + (size_t)ldh * c] : cmk<double2>(0.0, 0.0);
        hn = fmax(hn, cabs1(v));
        if (r == c) v = csub(v, m);
        A[e] = v;
    }
    red[lane] = hn;
    for (int r = lane; r < p; r += kHT) b[r] = cmk<double2>(1.0, 0.0);
    __syncthreads();
    if (lane == 0) {
        double t = 0.0;
        for (int q = 0; q < kHT; ++q) t = fmax(t, red[q]);
        red[0] = t;
    }
    __syncthreads();
    const double tiny = kEps * (red[0] > 0.0 ? red[0] : 1.0);
    // LU with row interchanges j <-> j+1
    for (int j = 0; j < p - 1; ++j) {
        double2 a = A[j * p + j], d = A[(j + 1) * p + j];
        const bool sw = cabs1(d) > cabs1(a);
        if (sw) { double2 t = a; a = d; d = t; }
        if (cabs1(a) == 0.0) a = cmk<double2>(tiny, 0.0);
        const double2 lm = cdiv(d, a);
        for (int c = j + lane; c < p; c += kHT) {
            double2 u = A[j * p + c], v = A[(j + 1) * p + c];
            if (sw) { double2 t = u; u = v; v = t; }
            if (c == j) u = a;
            A[j * p + c] = u;
            A[(j + 1) * p + c] = (c == j) ? cmk<double2>(0.0, 0.0) : csub(v, cmul(lm, u));
        }
        if (lane == 0) { piv[j] = sw ? 1 : 0; lmul[j] = lm; }
        __syncthreads();
    }
    if (lane == 0 && cabs1(A[(p - 1) * p + (p - 1)]) < tiny) A[(p - 1) * p + (p - 1)] = cmk<double2>(tiny, 0.0);
    __syncthreads();
    for (int it = 0; it < 2; ++it) {
        if (lane == 0) {
            // forward elimination on b, then back substitution (serial, O(p^2))
            for (int j = 0; j < p - 1; ++j) {
                if (piv[j]) { double2 t = b[j]; b[j] = b[j + 1]; b[j + 1] = t; }
                b[j + 1] = csub(b[j + 1], cmul(lmul[j], b[j]));
            }
            for (int r = p - 1; r >= 0; --r) {
                double2 acc = b[r];
                for (int c = r + 1; c < p; ++c) acc = csub(acc, cmul(A[r * p + c], b[c]));
                double2 dg = A[r * p + r];
                if (cabs1(dg) < tiny) dg = cmk<double2>(tiny, 0.0);
                b[r] = cdiv(acc, dg);
            }
            double n2 = 0.0;
            for (int r = 0; r < p; ++r) n2 += cabs2(b[r]);
            double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
            for (int r = 0; r < p; ++r) b[r] = cscale(b[r], inv);
        }
        __syncthreads();
    }
    for (int r = lane; r < p; r += kHT) Y[(size_t)sidx * p + r] = b[r];
}

}  // namespace

tsk_status hess_ritz_launch(const KryDesc* D, int count, int p, int k, double tol, bool full, hipStream_t s) {
    if (p < 1 || p > kMaxKrylov) return fail(TSK_EINVAL, "Hessenberg size must be in [1, 96]");
    size_t lds = size_t(p) * p * sizeof(double2);
    static bool attr_set = false;
    if (!attr_set) {
        const int mx = int(kMaxKrylov * kMaxKrylov * sizeof(double2));
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz<true>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz<false>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        TSK_HIP(hipFuncSetAttribute((const void*)k_ritz_coords, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        attr_set = true;
    }
    if (full)
        hipLaunchKernelGGL(k_hess_ritz<true>, dim3(count), dim3(kHT), lds, s, D, p, k, tol);
    else
        hipLaunchKernelGGL(k_hess_ritz<false>, dim3(count), dim3(kHT), lds, s, D, p, k, tol);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status ritz_coords_launch(const KryDesc* D, int count, int pmax, int k, hipStream_t s) {
    size_t lds = size_t(pmax) * pmax * sizeof(double2);
    hipLaunchKernelGGL(k_ritz_coords, dim3(k, count), dim3(kHT), lds, s, D);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

}  // namespace tsk
