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
// wait is just the LDS latency of one wave; inside the QR iteration, where the
// lanes exchange data only through LDS, the steps are ordered by
// wavefront-scope fences (wave_lds_sync) rather than workgroup barriers.
// T (p x p complex128, row-major) sits in LDS.  The deflation test of all subdiagonal entries is one ballot.
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
#include <cstring>
#include <type_traits>

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

// ---- wanted set (shared by the complex and the real eigensolver) ----------------------
// converged: res <= max(tol, res_floor |mu|); order by |mu| descending (ties:
// larger arg first, then index); skip unresolved copies; first k accepted.
__device__ inline void select_wanted(const double2* __restrict__ mu, const double* __restrict__ res,
                                     int* __restrict__ sel, RitzResult* __restrict__ rr, double* ctol, int* order,
                                     int* dupc, int p, int k, double tol, double dup_rel, double res_floor,
                                     int failed, int total, int lane) {
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

// FULLZ: accumulate all of Z (standalone use, every eigenvector formed);
// otherwise only the last row of Z is tracked (all the residuals need) and the
// wanted Ritz coordinates are computed afterwards by inverse iteration.
template <bool FULLZ>
__global__ __launch_bounds__(kHT) void k_hess_ritz(StepSet ss, int kreq, double tol) {
    const int p = ss.p[blockIdx.y];
    const int k = kreq < p ? kreq : p;
    const KryDesc& dsc = ss.tab[blockIdx.y][blockIdx.x];
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
    for (int e = lane; e < p * p; e += kHT) {  // H is column-major: consecutive lanes read down a column
        const int c = e / p, r = e % p;
        const double2 v = (r <= c + 1) ? H[r + (size_t)ldh * c] : cmk<double2>(0.0, 0.0);
        bad = bad || !isfinite(v.x) || !isfinite(v.y);
        T[r * p + c] = v;
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
        wave_lds_sync();
        if (l > 0 && lane == 0) T[l * p + (l - 1)] = cmk<double2>(0.0, 0.0);
        wave_lds_sync();
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
            wave_lds_sync();
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
        select_wanted(mu, res, sel, rr, ctol, order, dupc, p, k, tol, dup_rel, res_floor, failed, total, lane);
    }
}

// ---- real Hessenberg matrices (real operators) ------------------------------------------
// Francis double-shift QR in real arithmetic (Francis 1961; Golub & Van Loan,
// "Matrix Computations", Algorithms 7.5.1-7.5.2): each sweep chases a 3-element
// Householder bulge down the active window with shifts from the trailing 2x2
// block (an exceptional shift every tenth iteration), deflation on negligible
// subdiagonal entries, and every converged 2x2 block with real eigenvalues split
// by one rotation, so T ends quasi upper triangular with 2x2 blocks only for
// complex conjugate pairs.  The similarity P T P of one bulge step touches three
// rows and three columns whose only overlap is a 3x3 block.  A single wavefront
// issues one instruction every four cycles, so the sweep is bound by the
// instructions per bulge step: the sweep keeps the block, the entries near the
// bulge and each lane's window of Z in registers and runs each step as
// straight-line code (sweep_window), whether only the last row of Z is tracked
// (the Ritz analysis) or all of it (the Krylov-Schur contraction).  H = Z T
// Z^T; the eigenvector of each Ritz value follows by back substitution through the
// quasi-triangular T (one lane per eigenvalue, complex arithmetic for pairs).

// Householder vector for (x, y, z): v = (1, v1, v2), tau, with
// (I - tau v v^T) (x, y, z)^T = (alpha, 0, 0)^T.  tau = 0 when y = z = 0.  With
// rho = ||(x, y, z)||, alpha = -sign(x) rho, u0 = x - alpha: v = (y, z)/u0 and
// tau = |u0| / rho, so one reciprocal square root and one reciprocal suffice
// (hardware estimates refined by Newton steps; a plain path outside the range
// where the squares are safe).
__device__ inline double rcp_full(double v) {
    double y = __builtin_amdgcn_rcp(v);
    y = fma(y, fma(-v, y, 1.0), y);
    y = fma(y, fma(-v, y, 1.0), y);
    return y;
}

__device__ inline void house3(double x, double y, double z, double& v1, double& v2, double& tau, double& alpha) {
    const double sig = y * y + z * z;
    if (sig == 0.0) {
        v1 = v2 = tau = 0.0;
        alpha = x;
        return;
    }
    const double s2 = x * x + sig;
    if (s2 > 1e-280 && s2 < 1e280) {
        const double r = rsqrt_full(s2);  // 1 / rho
        const double rho = s2 * r;
        alpha = x >= 0.0 ? -rho : rho;
        const double u0 = x - alpha;  // no cancellation: x and -alpha share a sign
        const double iu = rcp_full(u0);
        v1 = y * iu;
        v2 = z * iu;
        tau = fabs(u0) * r;
        return;
    }
    const double rho = sqrt(s2);
    alpha = x >= 0.0 ? -rho : rho;
    const double u0 = x - alpha;
    v1 = y / u0;
    v2 = z / u0;
    tau = (alpha - x) / alpha;
}

__device__ inline double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Eigenvector z (complex, z[j] = 0 beyond the eigenvalue's block) of the quasi
// upper-triangular real T (row-major p x p) for eigenvalue index q with value m;
// blk[j]: 0 = 1x1, 1 = first / 2 = second row of a 2x2 block.  Returns ||z||^2.
__device__ inline double quasi_eigvec(const double* T, const int* blk, int p, int q, double2 m, double2* z) {
    double smin = kEps * (fabs(m.x) + fabs(m.y));
    if (smin < 1e-290) smin = 1e-290;
    int c;  // next row to solve (downwards to 0)
    double nrm = 1.0;
    if (blk[q] == 0) {
        z[q] = cmk<double2>(1.0, 0.0);
        c = q - 1;
    } else {
        // rows (r0, r0+1) of the pair; z[r0+1] = 1, z[r0] = (m - T[r0+1][r0+1]) / T[r0+1][r0]
        const int r0 = blk[q] == 1 ? q : q - 1;
        const double sub = T[(r0 + 1) * p + r0];
        const double2 z0 = cscale(cmk<double2>(m.x - T[(r0 + 1) * p + r0 + 1], m.y), 1.0 / sub);
        z[r0 + 1] = cmk<double2>(1.0, 0.0);
        z[r0] = z0;
        nrm += cabs2(z0);
        c = r0 - 1;
    }
    const int top = blk[q] == 1 ? q + 1 : q;  // last nonzero index
    while (c >= 0) {
        if (blk[c] == 2) {
            // 2x2 block (c-1, c): [T - m I] [z_{c-1}; z_c] = -[r_{c-1}; r_c]
            double2 r1 = cmk<double2>(0.0, 0.0), r2 = cmk<double2>(0.0, 0.0);
            for (int j = c + 1; j <= top; ++j) {
                r1 = cadd(r1, cscale(z[j], T[(c - 1) * p + j]));
                r2 = cadd(r2, cscale(z[j], T[c * p + j]));
            }
            const double2 a = cmk<double2>(T[(c - 1) * p + (c - 1)] - m.x, -m.y);
            const double2 b = cmk<double2>(T[(c - 1) * p + c], 0.0);
            const double2 d = cmk<double2>(T[c * p + (c - 1)], 0.0);
            const double2 e = cmk<double2>(T[c * p + c] - m.x, -m.y);
            double2 det = csub(cmul(a, e), cmul(b, d));
            if (cabs1(det) < smin) det = cmk<double2>(smin, 0.0);
            // Cramer's rule on -r
            const double2 x1 = cdiv(csub(cmul(b, r2), cmul(e, r1)), det);
            const double2 x2 = cdiv(csub(cmul(d, r1), cmul(a, r2)), det);
            z[c - 1] = x1;
            z[c] = x2;
            nrm += cabs2(x1) + cabs2(x2);
            c -= 2;
        } else {
            double2 r = cmk<double2>(0.0, 0.0);
            for (int j = c + 1; j <= top; ++j) r = cadd(r, cscale(z[j], T[c * p + j]));
            double2 den = cmk<double2>(T[c * p + c] - m.x, -m.y);
            if (cabs1(den) < smin) den = cmk<double2>(smin, 0.0);
            const double2 x = cdiv(cmk<double2>(-r.x, -r.y), den);
            z[c] = x;
            nrm += cabs2(x);
            c -= 1;
        }
    }
    for (int j = top + 1; j < p; ++j) z[j] = cmk<double2>(0.0, 0.0);
    return nrm;
}

// Rotation G = [[cs, sn], [-sn, cs]] applied as T <- G T G^T on indices (i, i+1)
// of the full matrix (rows i, i+1 from column cfrom; columns i, i+1 for rows
// 0..rto) and Z <- Z G^T: FZ = false, zl is the last row of Z; FZ = true, zl
// is all of Z (row-major p x p).  One wavefront, uniform control flow.
template <bool FZ>
__device__ inline void rot_similarity(double* T, double* zl, int p, int i, double cs, double sn, int cfrom, int rto,
                                      int lane) {
    for (int c = cfrom + lane; c < p; c += kHT) {
        const double u = T[i * p + c], v = T[(i + 1) * p + c];
        T[i * p + c] = cs * u + sn * v;
        T[(i + 1) * p + c] = -sn * u + cs * v;
    }
    wave_lds_sync();
    for (int r = lane; r <= rto; r += kHT) {
        const double u = T[r * p + i], v = T[r * p + i + 1];
        T[r * p + i] = cs * u + sn * v;
        T[r * p + i + 1] = -sn * u + cs * v;
    }
    if constexpr (FZ) {
        for (int r = lane; r < p; r += kHT) {
            const double u = zl[r * p + i], v = zl[r * p + i + 1];
            zl[r * p + i] = cs * u + sn * v;
            zl[r * p + i + 1] = -sn * u + cs * v;
        }
    } else if (lane == 0) {
        const double u = zl[i], v = zl[i + 1];
        zl[i] = cs * u + sn * v;
        zl[i + 1] = -sn * u + cs * v;
    }
    wave_lds_sync();
}

// One double-shift sweep over the active window l..ihi (ihi - l >= 2) with the
// state near the bulge in registers, and Z <- Z P_k: with FZ all of Z (zl, p x p
// row-major; lane i holds Z[i][k..k+2] and stores Z[i][k] after step k), else
// only its last row (zl, a window shared by every lane).
// The sweep applies T <- P_k T P_k for k = l..ihi-1 (3-element reflectors, then
// a 2-element one at k = ihi - 1).  Left and right products commute, so every
// entry outside the moving 3 x 3 block meets its updates in a fixed order: row
// r's entries in columns k..k+2 (r < k) get the right factor of step k, column
// c's entries in rows k..k+2 (c >= k + 3) the left factor.  Lane i (and i + 64
// when p > 64) holds a window of three such entries, T[i][k..k+2] while i < k
// and T[k..k+2][i] while i >= k + 3; both updates are w <- w - tau (v.w) v, so
// every lane runs the same instructions.  The block, the bulge (x, y, z), row
// k + 3 of the window (0, 0, T[k+3][k+2] before step k) and the window of zl are
// computed by every lane alike.  After step k an entry that no later step of the
// sweep changes in the same way goes to LDS (T[i][k] of a row window, T[k][i] of
// a column window, T[k][k], zl[k], the annihilated column k - 1); the next step
// takes column k + 3 (rows k..k+2) into the block and row k's new window entry
// from lane k + 3 by readlane, and every other entry it needs from LDS, where
// it is either untouched so far in this sweep or was stored at least one step
// earlier.  Per step: one reflector, one 3 x 3 two-sided update and one window
// update per lane, with no wait on LDS in the chain from one reflector to the
// next.
template <bool B> using bool_c = std::integral_constant<bool, B>;

template <int S, bool FZ>
__device__ inline void sweep_window(double* Tr, double* zl, int p, int l, int ihi, double x, double y, double z,
                                    int lane) {
    // sink[0] takes the stores of lanes with no window entry to store; sink[1]
    // stays 0 and is what those lanes load, so no lane branches on its role
    __shared__ double sink[2];
    if (lane == 0) sink[1] = 0.0;
    double B[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) B[a][b] = Tr[(l + a) * p + l + b];
    // the last row of Z (its window shared by every lane), or with FZ all of Z
    // (row-major p x p; lane i's window of row i, zr = &Z[i][k])
    double Z0 = 0.0, Z1 = 0.0, Z2 = 0.0;
    if constexpr (!FZ) {
        Z0 = zl[l];
        Z1 = zl[l + 1];
        Z2 = zl[l + 2];
    }
    double E2 = (l + 3 <= ihi) ? Tr[(l + 3) * p + l + 2] : 0.0;
    // lane window i: rp = &T[i][k] (row role, i < k), cp = &T[k][i] (column role,
    // i >= k + 3), both advanced with k
    double W[S][3];
    double* rp[S];
    double* cp[S];
    double ZW[FZ ? S : 1][3];
    double* zr[FZ ? S : 1];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int i = lane + kHT * s;
        rp[s] = Tr + i * p + l;
        cp[s] = Tr + l * p + i;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double* src = i < l ? rp[s] + a : (i >= l + 3 && i < p ? cp[s] + a * p : sink + 1);
            W[s][a] = *src;
        }
        if constexpr (FZ) {
            zr[s] = zl + i * p + l;
#pragma unroll
            for (int a = 0; a < 3; ++a) ZW[s][a] = *(i < p ? zr[s] + a : sink + 1);
        }
    }
    double* dg = Tr + l * p + l;  // &T[k][k]
    double* zp = zl + l;          // &zl[k]
    wave_lds_sync();
    // step k; THREE: a 3-element reflector (else the final 2-element one at
    // k = ihi - 1); NEXT3: step k + 1 has a 3-element reflector too
    auto step = [&](auto three_c, auto next3_c, int k) {
        constexpr bool THREE = decltype(three_c)::value;
        constexpr bool NEXT3 = decltype(next3_c)::value;
        // reflector P = I - tau v v^T, v = (1, v1, v2), P (x, y, z)^T = (alpha, 0, 0)^T.
        // With y = z = 0 and x != 0 the formulas give tau = 2 (P flips the sign of
        // row and column k), a valid reflector; only sums of squares outside the
        // safe range, x = y = z = 0 included, take the careful path.
        double v1, v2, tau, alpha;
        {
            const double zz = THREE ? z : 0.0;
            const double s2 = fma(x, x, fma(y, y, zz * zz));
            if (__builtin_amdgcn_readfirstlane((s2 > 1e-280 && s2 < 1e280) ? 1 : 0)) {
                const double r = rsqrt_full(s2);  // 1 / rho
                const double rho = s2 * r;
                alpha = x >= 0.0 ? -rho : rho;
                const double u0 = x - alpha;
                const double iu = rcp_full(u0);
                v1 = y * iu;
                v2 = zz * iu;
                tau = fabs(u0) * r;
            } else {
                house3(x, y, zz, v1, v2, tau, alpha);
            }
        }
        // block: B <- P B P = B - v a^T - b v^T, a = tau (B^T v - tau g v), b = tau B v, g = v^T B v
        {
            const double vv[3] = {1.0, v1, v2};
            double u[3], w[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                u[a] = fma(v2, B[a][2], fma(v1, B[a][1], B[a][0]));
                w[a] = fma(v2, B[2][a], fma(v1, B[1][a], B[0][a]));
            }
            const double tg = tau * fma(v2, u[2], fma(v1, u[1], u[0]));
            double av[3], bv[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                av[a] = tau * fma(-tg, vv[a], w[a]);
                bv[a] = tau * u[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) B[a][b] = fma(-bv[a], vv[b], fma(-vv[a], av[b], B[a][b]));
        }
        // row k + 3 (right factor; (0, 0, E2) before the step), zl, the lanes' windows
        const double te = tau * (v2 * E2);
        const double E0 = -te, E1 = -te * v1;
        E2 = fma(-te, v2, E2);
        if constexpr (FZ) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double tz = tau * fma(v2, ZW[s][2], fma(v1, ZW[s][1], ZW[s][0]));
                ZW[s][0] -= tz;
                ZW[s][1] = fma(-tz, v1, ZW[s][1]);
                ZW[s][2] = fma(-tz, v2, ZW[s][2]);
            }
        } else {
            const double tz = tau * fma(v2, Z2, fma(v1, Z1, Z0));
            Z0 -= tz;
            Z1 = fma(-tz, v1, Z1);
            Z2 = fma(-tz, v2, Z2);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const double tw = tau * fma(v2, W[s][2], fma(v1, W[s][1], W[s][0]));
            W[s][0] -= tw;
            W[s][1] = fma(-tw, v1, W[s][1]);
            W[s][2] = fma(-tw, v2, W[s][2]);
        }
        if (lane == 0) {
            if (k > l) {  // the reflector turned column k - 1 into (alpha, 0, 0)
                dg[-1] = alpha;
                dg[p - 1] = 0.0;
                if (THREE) dg[2 * p - 1] = 0.0;
            }
            dg[0] = B[0][0];
            if (!FZ) zp[0] = Z0;
            if (!THREE) {
                dg[1] = B[0][1];
                dg[p] = B[1][0];
                dg[p + 1] = B[1][1];
                if (!FZ) zp[1] = Z1;
            }
        }
        constexpr int NB = THREE ? 3 : 2;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = lane + kHT * s;
            const bool row = i < k, col = i >= k + NB && i < p;
            double* d0 = row ? rp[s] : (col ? cp[s] : sink);
            *d0 = W[s][0];
            if (!THREE) *(row ? d0 + 1 : (col ? d0 + p : sink)) = W[s][1];
            if constexpr (FZ) {  // Z[i][k] is final for the sweep
                double* zd = i < p ? zr[s] : sink;
                *zd = ZW[s][0];
                if (!THREE) *(i < p ? zd + 1 : sink) = ZW[s][1];
            }
        }
        if constexpr (THREE) {
            // keeps the LDS reads below after the stores above (other lanes read them)
            wave_lds_sync();
            const double xn = B[1][0], yn = B[2][0];
            double cB = 0.0, cC = 0.0, d33 = 0.0, e2n = 0.0, z2n = 0.0;
            if constexpr (NEXT3) {  // column k + 3 (k + 3 <= ihi) enters the block
                const int src = k + 3;
                double a1 = W[0][1], a2 = W[0][2];
                if constexpr (S > 1) {
                    if (src >= kHT) {
                        a1 = W[1][1];
                        a2 = W[1][2];
                    }
                }
                cB = readlane_d(a1, src % kHT);
                cC = readlane_d(a2, src % kHT);
                d33 = dg[3 * p + 3];
                e2n = *(k + 4 <= ihi ? dg + 4 * p + 3 : sink + 1);
                if (!FZ) z2n = zp[3];
            }
            const double b01 = B[0][1], b02 = B[0][2];
            B[0][0] = B[1][1];
            B[0][1] = B[1][2];
            B[0][2] = cB;
            B[1][0] = B[2][1];
            B[1][1] = B[2][2];
            B[1][2] = cC;
            B[2][0] = NEXT3 ? E1 : 0.0;
            B[2][1] = NEXT3 ? E2 : 0.0;
            B[2][2] = d33;
            // every lane shifts its window (the values of a lane without one are
            // never used); row k takes the block's row and T[k][k+3], which lane
            // k + 3 has just stored; the other rows and the columns load their new entry
            const int cfirst = k + 1 + (NEXT3 ? 3 : 2);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int i = lane + kHT * s;
                double nw = 0.0;
                if constexpr (NEXT3) {
                    const bool row = i <= k, col = i >= cfirst && i < p;
                    nw = *(row ? rp[s] + 3 : (col ? cp[s] + 3 * p : sink + 1));
                }
                const bool nr = i == k;
                W[s][0] = nr ? b01 : W[s][1];
                W[s][1] = nr ? b02 : W[s][2];
                W[s][2] = nw;
                rp[s] += 1;
                cp[s] += p;
                if constexpr (FZ) {  // Z[i][k+3] is untouched so far in the sweep
                    const int iz = lane + kHT * s;
                    ZW[s][0] = ZW[s][1];
                    ZW[s][1] = ZW[s][2];
                    ZW[s][2] = NEXT3 ? *(iz < p ? zr[s] + 3 : sink + 1) : 0.0;
                    zr[s] += 1;
                }
            }
            dg += p + 1;
            zp += 1;
            E2 = e2n;
            Z0 = Z1;
            Z1 = Z2;
            Z2 = z2n;
            x = xn;
            y = yn;
            z = NEXT3 ? E0 : 0.0;
        }
    };
    int k = l;
    for (; k <= ihi - 3; ++k) step(bool_c<true>{}, bool_c<true>{}, __builtin_amdgcn_readfirstlane(k));
    step(bool_c<true>{}, bool_c<false>{}, ihi - 2);
    step(bool_c<false>{}, bool_c<false>{}, ihi - 1);
}

// Francis double-shift QR of the p x p real Hessenberg matrix in Tr (row-major,
// LDS) to quasi upper-triangular form; blk marks the 2x2 blocks (1 = first, 2 =
// second row).  zl: last row of Z (FZ = false) or all of Z (FZ = true), updated
// with every transformation.  total: sweeps used; failed: no convergence
// within 30 max(p, 10) sweeps.
// stop (optional, host-written): the caller no longer needs this analysis; it
// is read once per sweep, one sweep ahead of its use so the load's latency
// hides behind the sweep, and a set flag ends the iteration with failed = 2.
__device__ inline int read_stop(const int* stop) {
    return stop ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0;
}

template <bool FZ>
__device__ __attribute__((always_inline)) inline void francis_real(double* Tr, double* zl, int* blk, int p, int lane,
                                                                   int& total, int& failed,
                                                                   const int* stop = nullptr) {
    int ihi = p - 1, its = 0;
    total = 0;
    failed = 0;
    const int itmax = 30 * (p > 10 ? p : 10);
    int stop_seen = read_stop(stop);
    while (ihi > 0) {
        if (__builtin_amdgcn_readfirstlane(stop_seen)) {
            failed = 2;
            break;
        }
        stop_seen = read_stop(stop);
        // deflation: largest l <= ihi with a negligible T[l][l-1] (else 0)
        bool s0 = false, s1 = false;
        {
            int i = lane + 1;
            if (i <= ihi) {
                double tst = fabs(Tr[(i - 1) * p + (i - 1)]) + fabs(Tr[i * p + i]);
                if (tst == 0.0) tst = 1.0;
                s0 = fabs(Tr[i * p + (i - 1)]) <= kEps * tst;
            }
            i = lane + 65;
            if (i <= ihi) {
                double tst = fabs(Tr[(i - 1) * p + (i - 1)]) + fabs(Tr[i * p + i]);
                if (tst == 0.0) tst = 1.0;
                s1 = fabs(Tr[i * p + (i - 1)]) <= kEps * tst;
            }
        }
        const unsigned long long m0 = __ballot(s0), m1 = __ballot(s1);
        const int l = m1 ? highest_bit(m1) + 65 : (m0 ? highest_bit(m0) + 1 : 0);
        wave_lds_sync();
        if (l > 0 && lane == 0) Tr[l * p + (l - 1)] = 0.0;
        wave_lds_sync();
        if (l == ihi) {  // 1x1 block converged
            --ihi;
            its = 0;
            continue;
        }
        if (l == ihi - 1) {  // 2x2 block: split when its eigenvalues are real
            const int i = ihi - 1;
            const double a = Tr[i * p + i], b = Tr[i * p + i + 1], c = Tr[(i + 1) * p + i], d = Tr[(i + 1) * p + i + 1];
            const double hp = 0.5 * (a - d);
            const double disc = hp * hp + b * c;
            if (disc >= 0.0) {
                // eigenvalue closest to d, eigenvector (lam - d, c) -> rotation taking it to e_1
                const double sq = sqrt(disc);
                const double lam = d + (hp >= 0.0 ? hp + sq : hp - sq);
                double ex = lam - d, ey = c;
                const double en = hypot(ex, ey);
                if (en > 0.0) {
                    const double cs = ex / en, sn = ey / en;
                    rot_similarity<FZ>(Tr, zl, p, i, cs, sn, i, i + 1, lane);
                }
                if (lane == 0) Tr[(i + 1) * p + i] = 0.0;
                wave_lds_sync();
            } else if (lane == 0) {
                blk[i] = 1;
                blk[i + 1] = 2;
            }
            wave_lds_sync();
            ihi -= 2;
            its = 0;
            continue;
        }
        if (++total > itmax) {
            failed = 1;
            break;
        }
        ++its;
        // double shift: s = sum, t = product of the trailing 2x2 eigenvalues
        double ss, tt;
        {
            const double a = Tr[(ihi - 1) * p + (ihi - 1)], b = Tr[(ihi - 1) * p + ihi];
            const double c = Tr[ihi * p + (ihi - 1)], d = Tr[ihi * p + ihi];
            if (its % 10 == 0) {
                const double sx = fabs(c) + fabs(Tr[(ihi - 1) * p + (ihi - 2)]);
                const double h11 = 0.75 * sx + d, h12 = -0.4375 * sx, h21 = sx;
                ss = 2.0 * h11;
                tt = h11 * h11 - h12 * h21;
            } else {
                ss = a + d;
                tt = a * d - b * c;
            }
        }
        double x, y, z;
        {
            const double t00 = Tr[l * p + l], t01 = Tr[l * p + l + 1], t10 = Tr[(l + 1) * p + l];
            const double t11 = Tr[(l + 1) * p + l + 1], t21 = Tr[(l + 2) * p + l + 1];
            x = t00 * t00 + t01 * t10 - ss * t00 + tt;
            y = t10 * (t00 + t11 - ss);
            z = t10 * t21;
        }
        if (p > kHT) sweep_window<2, FZ>(Tr, zl, p, l, ihi, x, y, z, lane);
        else sweep_window<1, FZ>(Tr, zl, p, l, ihi, x, y, z, lane);
        wave_lds_sync();
    }
}

// Ritz values of the quasi-triangular T (the 2x2 blocks give a + ib, a - ib in
// consecutive entries), eigenvectors of T in S (one per lane, back
// substitution) and residuals beta |zl . z_i| / ||z_i||, zl the last row of Z.
__device__ inline void real_ritz(const double* Tr, const int* blk, const double* zl, int p, double beta,
                                 double2* __restrict__ mu, double2* __restrict__ S, double* __restrict__ res, int lane) {
    for (int i = lane; i < p; i += kHT) {
        const double ti = Tr[i * p + i];
        double2 m = cmk<double2>(ti, 0.0);
        if (blk[i] != 0) {
            const int r0 = blk[i] == 1 ? i : i - 1;
            const double a = Tr[r0 * p + r0], b = Tr[r0 * p + r0 + 1], c = Tr[(r0 + 1) * p + r0];
            const double d = Tr[(r0 + 1) * p + r0 + 1];
            const double hp = 0.5 * (a - d);
            const double im = sqrt(fmax(-(hp * hp + b * c), 0.0));
            m = cmk<double2>(0.5 * (a + d), blk[i] == 1 ? im : -im);
        }
        mu[i] = m;
        double2* zc = S + (size_t)i * p;
        const double n2 = quasi_eigvec(Tr, blk, p, i, m, zc);
        double2 last = cmk<double2>(0.0, 0.0);
        for (int c = 0; c < p; ++c) last = cadd(last, cscale(zc[c], zl[c]));
        res[i] = fabs(beta) * cabs(last) / sqrt(n2);
    }
}

__global__ __launch_bounds__(kHT) void k_hess_ritz_real(StepSet ss, int kreq, double tol, int standalone) {
    const int p = ss.p[blockIdx.y];
    const int k = kreq < p ? kreq : p;
    const KryDesc& dsc = ss.tab[blockIdx.y][blockIdx.x];
    if (!dsc.active) return;
    const double2* __restrict__ H = dsc.H;
    const int ldh = dsc.ldh;
    double2* __restrict__ S = dsc.S;
    double2* __restrict__ mu = dsc.mu;
    double* __restrict__ res = dsc.res;
    int* __restrict__ sel = dsc.sel;
    RitzResult* __restrict__ rr = dsc.rr;
    extern __shared__ double Tr[];  // p*p, row-major
    __shared__ double zl[kMaxKrylov];
    __shared__ int blk[kMaxKrylov];
    __shared__ int order[kMaxKrylov];
    __shared__ int dupc[kMaxKrylov];
    __shared__ double ctol[kMaxKrylov];
    const int lane = threadIdx.x;

    const double beta = standalone ? dsc.scal[2] : H[p + (size_t)ldh * (p - 1)].x;
    bool bad = !isfinite(beta);
    for (int e = lane; e < p * p; e += kHT) {  // H is column-major: consecutive lanes read down a column
        const int c = e / p, r = e % p;
        const double v = (r <= c + 1) ? H[r + (size_t)ldh * c].x : 0.0;
        bad = bad || !isfinite(v);
        Tr[r * p + c] = v;
    }
    if (__ballot(bad)) {
        if (lane == 0 && rr) {
            rr->nonfinite = 1;
            rr->done = 0;
            rr->nsel = 0;
            rr->nconv = 0;
            rr->eig_fail = 0;
            rr->iters = 0;
        }
        return;
    }
    for (int c = lane; c < p; c += kHT) {
        zl[c] = c == p - 1 ? 1.0 : 0.0;
        blk[c] = 0;
    }
    __syncthreads();

    int total = 0, failed = 0;
    francis_real<false>(Tr, zl, blk, p, lane, total, failed, dsc.stop);
    if (failed == 2) return;  // a discarded step: nothing reads its outputs
    real_ritz(Tr, blk, zl, p, beta, mu, S, res, lane);
    __syncthreads();
    if (standalone) {
        if (lane == 0 && rr) {
            rr->eig_fail = failed;
            rr->iters = total;
        }
        return;
    }
    select_wanted(mu, res, sel, rr, ctol, order, dupc, p, k, tol, dsc.dup_rel, dsc.res_floor, failed, total, lane);
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
    for (int e = lane; e < p * p; e += kHT) {  // H is column-major: consecutive lanes read down a column
        const int c = e / p, r = e % p;
        double2 v = (r <= c + 1) ? H[r + (size_t)ldh * c] : cmk<double2>(0.0, 0.0);
        hn = fmax(hn, cabs1(v));
        if (r == c) v = csub(v, m);
        A[r * p + c] = v;
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
        // forward elimination on b (serial, O(p))
        if (lane == 0) {
            for (int j = 0; j < p - 1; ++j) {
                if (piv[j]) { double2 t = b[j]; b[j] = b[j + 1]; b[j + 1] = t; }
                b[j + 1] = csub(b[j + 1], cmul(lmul[j], b[j]));
            }
        }
        __syncthreads();
        // back substitution by columns: x_r = b_r / U_rr, then b_c -= U_cr x_r for
        // every c < r, one lane per c
        for (int r = p - 1; r >= 0; --r) {
            double2 dg = A[r * p + r];
            if (cabs1(dg) < tiny) dg = cmk<double2>(tiny, 0.0);
            const double2 xr = cdiv(b[r], dg);
            for (int c = lane; c < r; c += kHT) b[c] = csub(b[c], cmul(A[c * p + r], xr));
            if (lane == 0) b[r] = xr;
            __syncthreads();
        }
        double n2 = 0.0;
        for (int r = lane; r < p; r += kHT) n2 += cabs2(b[r]);
        red[lane] = n2;
        __syncthreads();
        if (lane == 0) {
            double t = 0.0;
            for (int q = 0; q < kHT; ++q) t += red[q];
            red[0] = t;
        }
        __syncthreads();
        const double inv = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
        for (int r = lane; r < p; r += kHT) b[r] = cscale(b[r], inv);
        __syncthreads();
    }
    for (int r = lane; r < p; r += kHT) Y[(size_t)sidx * p + r] = b[r];
}


// ---- Krylov-Schur contraction (Sec. 3.2.2, steps 2 to 4) --------------------------------
// After an expansion to order m the factorisation M V_m = V_m H_m + beta v_{m+1}
// e_m^T is analysed exactly as after an Arnoldi step (Ritz pairs, residuals,
// wanted set, stop test).  When the test fails, the contraction:
//  * real Schur form H_m = Z T Z^T (the Francis QR above, all of Z kept);
//  * kept set: the Ritz values with |mu| >= 1 - delta, at least k and at most
//    pmax of them, the leading ones in the wanted-set order, complex pairs whole;
//  * reordering of T so the kept blocks lead (swaps of adjacent diagonal blocks,
//    Z updated), which gives M (V Z) = (V Z) T + v_{m+1} (beta e_m^T Z), and the
//    truncation to the leading p columns: S = T_11, b = beta Z[m-1, 0:p];
//  * reduction of that Krylov-Schur decomposition to an equivalent Arnoldi one
//    (Stewart 2001: Krylov decompositions related by a similarity have the same
//    Ritz pairs): a reflector P0 with b^T P0 = beta' e_p^T, then reflectors that
//    leave e_p fixed and bring P0 S P0 to upper Hessenberg form from the bottom
//    row up.  The new basis is V_m W with W = Z[:, 0:p] P (m x p), the new
//    H_p is Hessenberg and H[p][p-1] = beta' >= 0, so the expansion continues
//    with plain Arnoldi steps from v_{p+1} = v_{m+1}.

// Swap of adjacent diagonal blocks of a real Schur form (Bai & Demmel 1993,
// direct swapping): A (N1 x N1) at j, B (N2 x N2) at j + N1, coupling C.  The
// solution X of A X - X B = C makes [-X; I] span B's invariant subspace of
// the (N1 + N2) block; the orthogonal Q of its QR factorisation moves B's
// eigenvalues first.  Refused (nothing changed, false) when the lower-left
// block of Q^T D Q is not negligible, which happens only for nearly equal
// eigenvalues.  Every lane solves the small problem itself (identical
// arithmetic, no broadcast); the updates of T's rows and columns and of Z's
// columns are split over the lanes.
template <int N1, int N2>
__device__ bool swap_blocks(double* Tr, double* Zf, int m, int j, int lane) {
    constexpr int NT = N1 + N2, K = N1 * N2;
    double D[NT][NT];
    double dnorm = 0.0;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            D[a][c] = Tr[(j + a) * m + j + c];
            dnorm = fmax(dnorm, fabs(D[a][c]));
        }
    // (I (x) A - B^T (x) I) vec X = vec C, unknown X[b][c] at index b + N1 c
    double G[K][K + 1];
#pragma unroll
    for (int e = 0; e < K; ++e)
#pragma unroll
        for (int u = 0; u <= K; ++u) G[e][u] = 0.0;
#pragma unroll
    for (int a = 0; a < N1; ++a)
#pragma unroll
        for (int c = 0; c < N2; ++c) {
            const int e = a + N1 * c;
#pragma unroll
            for (int b = 0; b < N1; ++b) G[e][b + N1 * c] += D[a][b];
#pragma unroll
            for (int d = 0; d < N2; ++d) G[e][a + N1 * d] -= D[N1 + d][N1 + c];
            G[e][K] = D[a][N1 + c];
        }
    double gmax = 0.0;
#pragma unroll
    for (int e = 0; e < K; ++e)
#pragma unroll
        for (int u = 0; u < K; ++u) gmax = fmax(gmax, fabs(G[e][u]));
    const double smin = fmax(kEps * gmax, 1e-290);
    // Gaussian elimination with partial pivoting (row exchanges by selects)
#pragma unroll
    for (int col = 0; col < K; ++col) {
#pragma unroll
        for (int r = col + 1; r < K; ++r)
            if (fabs(G[r][col]) > fabs(G[col][col])) {
#pragma unroll
                for (int u = 0; u <= K; ++u) {
                    const double t = G[r][u];
                    G[r][u] = G[col][u];
                    G[col][u] = t;
                }
            }
        if (fabs(G[col][col]) < smin) G[col][col] = smin;
#pragma unroll
        for (int r = col + 1; r < K; ++r) {
            const double f = G[r][col] / G[col][col];
#pragma unroll
            for (int u = col; u <= K; ++u) G[r][u] -= f * G[col][u];
        }
    }
    double x[K];
#pragma unroll
    for (int r = K - 1; r >= 0; --r) {
        double acc = G[r][K];
#pragma unroll
        for (int u = r + 1; u < K; ++u) acc -= G[r][u] * x[u];
        x[r] = acc / G[r][r];
    }
    // Householder QR of Y = [-X; I] (NT x N2), Q = H_0 H_1 ...
    double Y[NT][N2], Q[NT][NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
#pragma unroll
        for (int c = 0; c < N2; ++c) Y[a][c] = a < N1 ? -x[a + N1 * c] : (a - N1 == c ? 1.0 : 0.0);
#pragma unroll
        for (int c = 0; c < NT; ++c) Q[a][c] = a == c ? 1.0 : 0.0;
    }
#pragma unroll
    for (int c = 0; c < N2; ++c) {
        double sig = 0.0;
#pragma unroll
        for (int r = c + 1; r < NT; ++r) sig += Y[r][c] * Y[r][c];
        if (sig == 0.0) continue;
        const double y0 = Y[c][c];
        const double rho = sqrt(y0 * y0 + sig);
        const double al = y0 >= 0.0 ? -rho : rho;
        const double tau = (al - y0) / al;
        double v[NT];
#pragma unroll
        for (int r = 0; r < NT; ++r) v[r] = r < c ? 0.0 : (r == c ? 1.0 : Y[r][c] / (y0 - al));
#pragma unroll
        for (int q = c; q < N2; ++q) {
            double d = 0.0;
#pragma unroll
            for (int r = c; r < NT; ++r) d += v[r] * Y[r][q];
#pragma unroll
            for (int r = c; r < NT; ++r) Y[r][q] -= tau * d * v[r];
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            double d = 0.0;
#pragma unroll
            for (int r = c; r < NT; ++r) d += Q[a][r] * v[r];
#pragma unroll
            for (int r = c; r < NT; ++r) Q[a][r] -= tau * d * v[r];
        }
    }
    // test the swapped block: lower-left N1 x N2 of Q^T D Q must be negligible
    const double thresh = fmax(20.0 * kEps * dnorm, 1e-290);
    bool ok = true;
#pragma unroll
    for (int a = N2; a < NT; ++a)
#pragma unroll
        for (int c = 0; c < N2; ++c) {
            double t = 0.0;
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                double dq = 0.0;
#pragma unroll
                for (int q = 0; q < NT; ++q) dq += D[r][q] * Q[q][c];
                t += Q[r][a] * dq;
            }
            ok = ok && fabs(t) <= thresh;
        }
    __syncthreads();  // every lane has read D
    if (!ok) return false;
    for (int c = j + lane; c < m; c += kHT) {  // rows j.. of T: Q^T T
        double t[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) t[a] = Tr[(j + a) * m + c];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < NT; ++r) acc += Q[r][a] * t[r];
            Tr[(j + a) * m + c] = acc;
        }
    }
    __syncthreads();
    for (int r = lane; r < m; r += kHT) {  // columns j.. of T (rows < j + NT) and of Z: T Q, Z Q
        double t[NT], z[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            t[a] = r < j + NT ? Tr[r * m + j + a] : 0.0;
            z[a] = Zf[r * m + j + a];
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            double at = 0.0, az = 0.0;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                at += t[q] * Q[q][a];
                az += z[q] * Q[q][a];
            }
            if (r < j + NT) Tr[r * m + j + a] = at;
            Zf[r * m + j + a] = az;
        }
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int a = N2; a < NT; ++a)
#pragma unroll
            for (int c = 0; c < N2; ++c) Tr[(j + a) * m + j + c] = 0.0;
    }
    __syncthreads();
    return true;
}

__device__ inline bool swap_at(double* Tr, double* Zf, int m, int j, int n1, int n2, int lane) {
    if (n1 == 1) return n2 == 1 ? swap_blocks<1, 1>(Tr, Zf, m, j, lane) : swap_blocks<1, 2>(Tr, Zf, m, j, lane);
    return n2 == 1 ? swap_blocks<2, 1>(Tr, Zf, m, j, lane) : swap_blocks<2, 2>(Tr, Zf, m, j, lane);
}

// Householder reflector P = I - tau v v^T on coordinates 0..len-1 with
// P x = alpha e_{len-1}, x = hv[0..len-1]; v (v[len-1] = 1) overwrites hv.
// tau = 0 (P = I, alpha = x[len-1]) when x[0..len-2] = 0.  One lane.
__device__ inline void house_last(double* hv, int len, double& tau, double& alpha) {
    const double xl = hv[len - 1];
    double sig = 0.0;
    for (int i = 0; i < len - 1; ++i) sig += hv[i] * hv[i];
    hv[len - 1] = 1.0;
    if (sig == 0.0) {
        tau = 0.0;
        alpha = xl;
        return;
    }
    const double rho = sqrt(xl * xl + sig);
    alpha = xl >= 0.0 ? -rho : rho;
    const double u = xl - alpha;
    for (int i = 0; i < len - 1; ++i) hv[i] /= u;
    tau = (alpha - xl) / alpha;
}

// S <- P S P for the leading kp x kp block S of Tr and Z[:, 0:len] <- Z[:, 0:len] P,
// P the reflector (hv, tau) on coordinates 0..len-1.
__device__ inline void reflect_both(double* Tr, double* Zf, int m, int kp, int len, const double* hv, double tau,
                                    int lane) {
    if (tau != 0.0) {
        for (int r = lane; r < m; r += kHT) {  // right factor: rows of S and of Z
            if (r < kp) {
                double d = 0.0;
                for (int c = 0; c < len; ++c) d += Tr[r * m + c] * hv[c];
                d *= tau;
                for (int c = 0; c < len; ++c) Tr[r * m + c] -= d * hv[c];
            }
            double d = 0.0;
            for (int c = 0; c < len; ++c) d += Zf[r * m + c] * hv[c];
            d *= tau;
            for (int c = 0; c < len; ++c) Zf[r * m + c] -= d * hv[c];
        }
        __syncthreads();
        for (int c = lane; c < kp; c += kHT) {  // left factor: columns of S
            double d = 0.0;
            for (int r = 0; r < len; ++r) d += hv[r] * Tr[r * m + c];
            d *= tau;
            for (int r = 0; r < len; ++r) Tr[r * m + c] -= d * hv[r];
        }
    }
    __syncthreads();
}

// contract: 0 = analysis only; 1 = contract unless the stop test is met;
// 2 = contract unconditionally (standalone use).  Skips an instance whose
// expansion broke down (rr->bd_step set: the host analyses that order).
// Outputs: mu, res, sel, rr as k_hess_ritz_real; on contraction rr->kept = p,
// rr->beta = beta', H rewritten ((m+1) x m, zero outside the new H_p and
// H[p][p-1]) and ksW = W (m x p, column-major).  rr->eig_fail = 2 when the
// reordering left no room for an expansion (p > m - 1).
__global__ __launch_bounds__(kHT) void k_ks_contract(const KryDesc* __restrict__ Dv, int m, int k, double tol,
                                                     int contract) {
    const KryDesc& dsc = Dv[blockIdx.x];
    if (!dsc.active) return;
    RitzResult* __restrict__ rr = dsc.rr;
    if (rr->bd_step) return;
    double2* __restrict__ H = dsc.H;
    const int ldh = dsc.ldh;
    extern __shared__ double lds[];
    double* Tr = lds;          // T, m x m row-major
    double* Zf = lds + m * m;  // Z, m x m row-major
    __shared__ int blk[kMaxKrylov];
    __shared__ int order[kMaxKrylov];
    __shared__ int dupc[kMaxKrylov];
    __shared__ int keep[kMaxKrylov];
    __shared__ double ctol[kMaxKrylov];
    __shared__ double hv[kMaxKrylov];
    __shared__ double sh_tau, sh_alpha;
    __shared__ int sh_go, sh_kp;
    const int lane = threadIdx.x;

    const double beta = H[m + (size_t)ldh * (m - 1)].x;
    bool bad = !isfinite(beta);
    for (int e = lane; e < m * m; e += kHT) {  // H is column-major: consecutive lanes read down a column
        const int c = e / m, r = e % m;
        const double v = (r <= c + 1) ? H[r + (size_t)ldh * c].x : 0.0;
        bad = bad || !isfinite(v);
        Tr[r * m + c] = v;
        Zf[e] = r == c ? 1.0 : 0.0;
    }
    if (__ballot(bad)) {
        if (lane == 0) {
            rr->nonfinite = 1;
            rr->done = 0;
            rr->nsel = 0;
            rr->nconv = 0;
            rr->eig_fail = 0;
            rr->iters = 0;
            rr->kept = 0;
        }
        return;
    }
    for (int c = lane; c < m; c += kHT) blk[c] = 0;
    __syncthreads();
    int total = 0, failed = 0;
    francis_real<true>(Tr, Zf, blk, m, lane, total, failed);
    __syncthreads();
    real_ritz(Tr, blk, Zf + (size_t)(m - 1) * m, m, beta, dsc.mu, dsc.S, dsc.res, lane);
    __syncthreads();
    select_wanted(dsc.mu, dsc.res, dsc.sel, rr, ctol, order, dupc, m, k, tol, dsc.dup_rel, dsc.res_floor, failed,
                  total, lane);
    __syncthreads();
    if (lane == 0) {
        sh_go = (contract == 2 || (contract == 1 && !rr->done)) && !failed;
        rr->kept = 0;
        if (sh_go) {  // kept count: |mu| >= 1 - delta, raised to k, lowered to pmax
            int pd = 0;
            for (int i = 0; i < m; ++i) pd += cabs(dsc.mu[i]) >= 1.0 - dsc.ks_delta ? 1 : 0;
            sh_kp = min(max(pd, k), dsc.ks_pmax);
        }
    }
    __syncthreads();
    if (!sh_go) return;
    for (int t = lane; t < m; t += kHT) keep[order[t]] = t < sh_kp ? 1 : 0;
    __syncthreads();
    if (lane == 0)  // complex pairs are kept whole
        for (int i = 0; i + 1 < m; ++i)
            if (blk[i] == 1 && (keep[i] | keep[i + 1])) keep[i] = keep[i + 1] = 1;
    __syncthreads();

    // reorder: every kept block moves up to the end of the kept region; a
    // refused swap keeps the blocks it could not pass as well
    int ks = 0, i = 0;
    while (i < m) {
        const int sz = blk[i] == 1 ? 2 : 1;
        if (keep[i]) {
            int pos = i;
            while (pos > ks) {
                const int sa = blk[pos - 1] == 2 ? 2 : 1;
                if (!swap_at(Tr, Zf, m, pos - sa, sa, sz, lane)) break;
                if (lane == 0) {
                    const int q = pos - sa;
                    for (int a = 0; a < sz; ++a) {
                        blk[q + a] = sz == 2 ? 1 + a : 0;
                        keep[q + a] = 1;
                    }
                    for (int a = 0; a < sa; ++a) {
                        blk[q + sz + a] = sa == 2 ? 1 + a : 0;
                        keep[q + sz + a] = 0;
                    }
                }
                __syncthreads();
                pos -= sa;
            }
            ks = pos + sz;
        }
        i += sz;
    }
    const int kp = ks;
    if (kp > m - 1) {
        if (lane == 0) rr->eig_fail = 2;
        return;
    }

    // Krylov-Schur decomposition of order kp -> Arnoldi form
    for (int c = lane; c < kp; c += kHT) hv[c] = beta * Zf[(size_t)(m - 1) * m + c];
    __syncthreads();
    if (lane == 0) {
        double tau, al;
        house_last(hv, kp, tau, al);
        sh_tau = tau;
        sh_alpha = al;
    }
    __syncthreads();
    double bnew = sh_alpha;  // b^T P0 = bnew e_kp^T
    reflect_both(Tr, Zf, m, kp, kp, hv, sh_tau, lane);
    for (int r0 = kp - 1; r0 >= 2; --r0) {
        for (int c = lane; c < r0; c += kHT) hv[c] = Tr[r0 * m + c];
        __syncthreads();
        if (lane == 0) {
            double tau, al;
            house_last(hv, r0, tau, al);
            sh_tau = tau;
            sh_alpha = al;
        }
        __syncthreads();
        const double al = sh_alpha;
        reflect_both(Tr, Zf, m, kp, r0, hv, sh_tau, lane);
        if (lane == 0) {
            for (int c = 0; c < r0 - 1; ++c) Tr[r0 * m + c] = 0.0;
            Tr[r0 * m + r0 - 1] = al;
        }
        __syncthreads();
    }
    if (bnew < 0.0) {  // similarity with diag(1, ..., 1, -1) makes beta' >= 0
        bnew = -bnew;
        for (int c = lane; c < kp - 1; c += kHT) {
            Tr[(kp - 1) * m + c] = -Tr[(kp - 1) * m + c];
            Tr[c * m + kp - 1] = -Tr[c * m + kp - 1];
        }
        for (int r = lane; r < m; r += kHT) Zf[r * m + kp - 1] = -Zf[r * m + kp - 1];
        __syncthreads();
    }
    for (int e = lane; e < ldh * m; e += kHT) {
        const int r = e % ldh, c = e / ldh;
        double v = 0.0;
        if (c < kp) {
            if (r < kp && r <= c + 1) v = Tr[r * m + c];
            else if (r == kp && c == kp - 1) v = bnew;
        }
        H[e] = cmk<double2>(v, 0.0);
    }
    double* __restrict__ W = dsc.ksW;
    for (int e = lane; e < m * kp; e += kHT) {
        const int r = e % m, c = e / m;
        W[e] = Zf[r * m + c];
    }
    if (lane == 0) {
        rr->kept = kp;
        rr->beta = bnew;
    }
}


// ---- symmetric tridiagonal matrices (Lanczos on M^dagger M) ------------------------------
// Ritz analysis of the Lanczos tridiagonal T_p: diagonal d_i = H[i][i], off-diagonal
// e_i = H[i+1][i] (the Lanczos beta), residual scale beta_p = H[p][p-1] (Sec. 3.3.2:
// for the symmetric M^dagger M the Hessenberg matrix becomes tridiagonal).  Implicit
// symmetric QR with the Wilkinson shift (Golub & Van Loan, "Matrix Computations",
// Algorithms 8.3.2-8.3.3): deflation on negligible e_i, each sweep a chase of Givens
// rotations down the active block.  The chase is a scalar recurrence, so lane 0
// runs it with d and e in LDS and records the rotations; every lane then applies
// them to its rows of Z (all eigenvectors, p x p in LDS).  Outputs as the Hessenberg
// solver: mu = (theta, 0), residual |beta_p Z[p-1][i]|, wanted set; and the unit Ritz
// coordinates of the wanted values (columns of Z) in S[s*p + r], so the Ritz vectors
// of the final step need no inverse iteration.
__global__ __launch_bounds__(kHT) void k_tridiag_ritz(StepSet ss, int kreq, double tol) {
    const int p = ss.p[blockIdx.y];
    const int k = kreq < p ? kreq : p;
    const KryDesc& dsc = ss.tab[blockIdx.y][blockIdx.x];
    if (!dsc.active) return;
    const double2* __restrict__ H = dsc.H;
    const int ldh = dsc.ldh;
    RitzResult* __restrict__ rr = dsc.rr;
    extern __shared__ double Zs[];  // p x p row-major
    __shared__ double d[kMaxKrylov], e[kMaxKrylov], rc[kMaxKrylov], rs[kMaxKrylov];
    __shared__ int order[kMaxKrylov];
    __shared__ int dupc[kMaxKrylov];
    __shared__ double ctol[kMaxKrylov];
    __shared__ int sh_l;
    const int lane = threadIdx.x;

    const double beta = H[p + (size_t)ldh * (p - 1)].x;
    bool bad = !isfinite(beta);
    for (int i = lane; i < p; i += kHT) {
        d[i] = H[i + (size_t)ldh * i].x;
        e[i] = i + 1 < p ? H[i + 1 + (size_t)ldh * i].x : 0.0;
        bad = bad || !isfinite(d[i]) || !isfinite(e[i]);
    }
    if (__ballot(bad)) {
        if (lane == 0) {
            rr->nonfinite = 1;
            rr->done = 0;
            rr->nsel = 0;
            rr->nconv = 0;
            rr->eig_fail = 0;
            rr->iters = 0;
        }
        return;
    }
    for (int t = lane; t < p * p; t += kHT) Zs[t] = (t / p == t % p) ? 1.0 : 0.0;
    __syncthreads();

    int hi = p - 1, total = 0, failed = 0;
    const int itmax = 30 * (p > 10 ? p : 10);
    while (hi > 0) {
        if (lane == 0) {  // active block [l, hi]: e[l..hi-1] not negligible
            int l = hi;
            while (l > 0) {
                if (fabs(e[l - 1]) <= kEps * (fabs(d[l - 1]) + fabs(d[l]))) {
                    e[l - 1] = 0.0;
                    break;
                }
                --l;
            }
            sh_l = l;
        }
        __syncthreads();
        const int l = sh_l;
        if (l == hi) {
            --hi;
            continue;
        }
        if (++total > itmax) {
            failed = 1;
            break;
        }
        if (lane == 0) {
            // Wilkinson shift: the eigenvalue of the trailing 2x2 block closer to d[hi]
            const double a = d[hi - 1], b = e[hi - 1], c = d[hi];
            const double del = 0.5 * (a - c);
            const double den = del + (del >= 0.0 ? 1.0 : -1.0) * sqrt(del * del + b * b);
            const double mu = den != 0.0 ? c - b * b / den : c;
            double x = d[l] - mu, z = e[l], bulge = 0.0;
            for (int kk = l; kk < hi; ++kk) {
                if (kk > l) {
                    x = e[kk - 1];
                    z = bulge;
                }
                const double r = sqrt(x * x + z * z);
                const double cs = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? z / r : 0.0;
                if (kk > l) e[kk - 1] = r;
                const double dk = d[kk], ek = e[kk], dk1 = d[kk + 1];
                d[kk] = cs * cs * dk + 2.0 * cs * sn * ek + sn * sn * dk1;
                d[kk + 1] = sn * sn * dk - 2.0 * cs * sn * ek + cs * cs * dk1;
                e[kk] = cs * sn * (dk1 - dk) + (cs * cs - sn * sn) * ek;
                if (kk + 1 < hi) {
                    bulge = sn * e[kk + 1];
                    e[kk + 1] = cs * e[kk + 1];
                }
                rc[kk] = cs;
                rs[kk] = sn;
            }
        }
        __syncthreads();
        for (int r = lane; r < p; r += kHT) {  // Z <- Z G^T, rotation by rotation
            double* zr = Zs + r * p;
            for (int kk = l; kk < hi; ++kk) {
                const double u = zr[kk], v = zr[kk + 1];
                zr[kk] = rc[kk] * u + rs[kk] * v;
                zr[kk + 1] = -rs[kk] * u + rc[kk] * v;
            }
        }
        __syncthreads();
    }
    double2* __restrict__ mu = dsc.mu;
    double* __restrict__ res = dsc.res;
    for (int i = lane; i < p; i += kHT) {
        mu[i] = cmk<double2>(d[i], 0.0);
        res[i] = fabs(beta) * fabs(Zs[(p - 1) * p + i]);
    }
    __syncthreads();
    select_wanted(mu, res, dsc.sel, rr, ctol, order, dupc, p, k, tol, dsc.dup_rel, dsc.res_floor, failed, total,
                  lane);
    __syncthreads();
    const int nsel = rr->nsel;
    for (int t = lane; t < nsel * p; t += kHT) {
        const int s = t / p, r = t % p;
        dsc.S[t] = cmk<double2>(Zs[r * p + dsc.sel[s]], 0.0);
    }
}

}  // namespace

tsk_status hess_ritz_launch(const KryDesc* D, int count, int p, int k, double tol, bool full, hipStream_t s,
                            bool real_h, bool attrs_only) {
    if (p < 1 || p > kMaxKrylov) return fail(TSK_EINVAL, "Hessenberg size must be in [1, 96]");
    static bool attr_set = false;
    if (!attr_set) {
        const int mx = int(kMaxKrylov * kMaxKrylov * sizeof(double2));
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz<true>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz<false>, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        TSK_HIP(hipFuncSetAttribute((const void*)k_ritz_coords, hipFuncAttributeMaxDynamicSharedMemorySize, mx));
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz_real, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(kMaxKrylov * kMaxKrylov * sizeof(double))));
        attr_set = true;
    }
    if (attrs_only) return TSK_OK;
    StepSet one{};
    one.tab[0] = D;
    one.p[0] = p;
    if (real_h) {
        // full: the standalone entry point (beta from scal[2]; values and residuals only)
        hipLaunchKernelGGL(k_hess_ritz_real, dim3(count, 1), dim3(kHT), size_t(p) * p * sizeof(double), s, one, k,
                           tol, full ? 1 : 0);
    } else {
        const size_t lds = size_t(p) * p * sizeof(double2);
        if (full)
            hipLaunchKernelGGL(k_hess_ritz<true>, dim3(count, 1), dim3(kHT), lds, s, one, k, tol);
        else
            hipLaunchKernelGGL(k_hess_ritz<false>, dim3(count, 1), dim3(kHT), lds, s, one, k, tol);
    }
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status ritz_steps_launch(const StepSet& ss, int n, int count, int k, double tol, bool svd, bool real_h,
                             hipStream_t s) {
    if (n < 1 || n > StepSet::kMax) return fail(TSK_EINVAL, "step batch size out of range");
    int pmax = 0;
    for (int i = 0; i < n; ++i) {
        if (ss.p[i] < 1 || ss.p[i] > kMaxKrylov) return fail(TSK_EINVAL, "Krylov order must be in [1, 96]");
        pmax = ss.p[i] > pmax ? ss.p[i] : pmax;
    }
    if (svd) return tridiag_ritz_launch_steps(ss, n, count, pmax, k, tol, s);
    TSK_TRY(hess_ritz_launch(ss.tab[0], count, ss.p[0], k, tol, false, s, real_h, /*attrs_only=*/true));
    if (real_h)
        hipLaunchKernelGGL(k_hess_ritz_real, dim3(count, n), dim3(kHT), size_t(pmax) * pmax * sizeof(double), s, ss,
                           k, tol, 0);
    else
        hipLaunchKernelGGL(k_hess_ritz<false>, dim3(count, n), dim3(kHT), size_t(pmax) * pmax * sizeof(double2), s,
                           ss, k, tol);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status tridiag_ritz_launch_steps(const StepSet& ss, int n, int count, int pmax, int k, double tol,
                                     hipStream_t s) {
    if (pmax < 1 || pmax > kMaxKrylov) return fail(TSK_EINVAL, "Lanczos order must be in [1, 96]");
    static bool attr_set = false;
    if (!attr_set) {
        TSK_HIP(hipFuncSetAttribute((const void*)k_tridiag_ritz, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(kMaxKrylov * kMaxKrylov * sizeof(double))));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_tridiag_ritz, dim3(count, n), dim3(kHT), size_t(pmax) * pmax * sizeof(double), s, ss, k,
                       tol);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status tridiag_ritz_launch(const KryDesc* D, int count, int p, int k, double tol, hipStream_t s) {
    StepSet one{};
    one.tab[0] = D;
    one.p[0] = p;
    return tridiag_ritz_launch_steps(one, 1, count, p, k, tol, s);
}

tsk_status ks_contract_launch(const KryDesc* D, int m, int k, double tol, int contract, hipStream_t s, int count) {
    if (m < 2 || m > kMaxKrylov) return fail(TSK_EINVAL, "Krylov-Schur order must be in [2, 96]");
    static bool attr_set = false;
    if (!attr_set) {
        TSK_HIP(hipFuncSetAttribute((const void*)k_ks_contract, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(2 * kMaxKrylov * kMaxKrylov * sizeof(double))));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_ks_contract, dim3(count), dim3(kHT), size_t(2) * m * m * sizeof(double), s, D, m, k, tol,
                       contract);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

namespace {
// Real H (column-major, ldh) into the real parts of the (m+1) x m complex
// layout the contraction reads, beta at (m, m-1); and the real parts back.
__global__ void k_pack_real(const double* __restrict__ H, int ldh, int m, double beta, double2* __restrict__ Hc) {
    for (int e = threadIdx.x; e < (m + 1) * m; e += blockDim.x) {
        const int r = e % (m + 1), c = e / (m + 1);
        const double v = r < m ? ((r <= c + 1) ? H[r + size_t(ldh) * c] : 0.0) : (c == m - 1 ? beta : 0.0);
        Hc[e] = cmk<double2>(v, 0.0);
    }
}
__global__ void k_unpack_real(const double2* __restrict__ Hc, int n, double* __restrict__ out) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) out[e] = Hc[e].x;
}
}  // namespace

tsk_status ks_contract_standalone(const double* H, int ldh, int m, double beta, int k, double delta, int pmax,
                                  void* mu, double* res, double* Hnew, double* W, int* kept, double* beta_new,
                                  hipStream_t s) {
    DevBuf Hc, S, sel, rr, dd;
    TSK_TRY(Hc.ensure(size_t(m + 1) * m * sizeof(double2)));
    TSK_TRY(S.ensure(size_t(m) * m * sizeof(double2)));
    TSK_TRY(sel.ensure(size_t(m) * sizeof(int)));
    TSK_TRY(rr.ensure(sizeof(RitzResult)));
    TSK_TRY(dd.ensure(sizeof(KryDesc)));
    KryDesc d;
    std::memset(&d, 0, sizeof(d));
    d.H = Hc.as<double2>();
    d.ldh = m + 1;
    d.S = S.as<double2>();
    d.mu = static_cast<double2*>(mu);
    d.res = res;
    d.sel = sel.as<int>();
    d.rr = rr.as<RitzResult>();
    d.active = 1;
    d.ksW = W;
    d.ks_delta = delta;
    d.ks_pmax = pmax;
    RitzResult r0{};
    hipLaunchKernelGGL(k_pack_real, dim3(1), dim3(256), 0, s, H, ldh, m, beta, d.H);
    TSK_HIP(hipMemcpyAsync(rr.ptr, &r0, sizeof(r0), hipMemcpyHostToDevice, s));
    TSK_HIP(hipMemcpyAsync(dd.ptr, &d, sizeof(d), hipMemcpyHostToDevice, s));
    TSK_TRY(ks_contract_launch(dd.as<KryDesc>(), m, k, 0.0, 2, s));
    hipLaunchKernelGGL(k_unpack_real, dim3(1), dim3(256), 0, s, d.H, (m + 1) * m, Hnew);
    RitzResult h{};
    TSK_HIP(hipMemcpyAsync(&h, rr.ptr, sizeof(RitzResult), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    if (h.nonfinite) return fail(TSK_ENONFINITE, "H or beta is not finite");
    if (h.eig_fail) return fail(TSK_EEIG, h.eig_fail == 2 ? "Schur reordering left no room to expand"
                                                          : "Hessenberg QR did not converge");
    *kept = h.kept;
    *beta_new = h.beta;
    return TSK_OK;
}

tsk_status ritz_coords_launch(const KryDesc* D, int count, int pmax, int k, hipStream_t s) {
    size_t lds = size_t(pmax) * pmax * sizeof(double2);
    hipLaunchKernelGGL(k_ritz_coords, dim3(k, count), dim3(kHT), lds, s, D);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

}  // namespace tsk
