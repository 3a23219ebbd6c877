// Device-side Ritz analysis of the Arnoldi Hessenberg matrix (one workgroup).
//
// Ritz pairs (mu_H, y) of H_p give the approximations (mu, V_p y) of the
// eigenpairs of M (Sec. 3.2.1, eq. "m-step Arnoldi" and the Ritz relation that
// follows it); each pair is judged by |beta e_p^T y| (Sec. 3.2.2, eq. "Krylov
// convergence").  The eigensolver is the shifted QR algorithm on the Hessenberg
// matrix in complex arithmetic (Francis 1961; Golub & Van Loan, "Matrix
// Computations", Sec. 7.5): Wilkinson shift from the trailing 2x2 block,
// exceptional shifts every tenth iteration, deflation on negligible subdiagonal
// entries, Givens rotations accumulated into Z so that H = Z T Z^H with T upper
// triangular.  Eigenvectors of T by back substitution (swept column by column
// so the whole workgroup works on all eigenvectors at once), y = Z z, unit
// 2-norm.  A real H (real operators) is treated as complex; its conjugate
// pairs come out to rounding.
//
// The wanted set follows the stop rule documented with tsk_arnoldi: sort by
// |mu| descending (ties: larger arg mu first), accept converged values, skip an
// unconverged value that lies within its residual of a converged or an already
// accepted value, accept the rest; done when the first k accepted are converged.
//
// Layout: T (p x p complex128) in LDS, row-major T[r * p + c]; Z, the
// eigenvector sweep and Y in global scratch, column-major [col * p + row].
#include "ops.hpp"

namespace tsk {

namespace {

constexpr int kHT = 256;  // threads of the eigensolver workgroup
constexpr double kEps = 2.220446049250313e-16;

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

// Givens rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0], c real.
__device__ inline void givens(double2 x, double2 y, double& c, double2& s) {
    double ax = cabs(x), ay = cabs(y);
    if (ay == 0.0) { c = 1.0; s = cmk<double2>(0.0, 0.0); return; }
    if (ax == 0.0) {  // swap rows: G = [[0, conj(y)/|y|], [-(y/|y|), 0]]
        c = 0.0;
        s = cmk<double2>(y.x / ay, -y.y / ay);
        return;
    }
    double rho = hypot(ax, ay);
    c = ax / rho;
    double2 ph = cmk<double2>(x.x / ax, x.y / ax);              // x/|x|
    s = cscale(cmul(ph, cmk<double2>(y.x, -y.y)), 1.0 / rho);  // (x/|x|) conj(y) / rho
}

__global__ __launch_bounds__(kHT) void k_hess_ritz(const double2* __restrict__ H, int ldh, int p,
                                                  const double* __restrict__ beta_dev, double beta_val,
                                                  double2* __restrict__ Z, double2* __restrict__ S,
                                                  double2* __restrict__ mu, double2* __restrict__ Y,
                                                  double* __restrict__ res, int k, double tol, double T,
                                                  int* __restrict__ sel, RitzResult* __restrict__ rr) {
    extern __shared__ double2 Tl[];  // p*p
    __shared__ double sh_c;
    __shared__ double2 sh_s;
    __shared__ int sh_l, sh_ihi, sh_fail, sh_iters;
    __shared__ double2 sh_shift;
    __shared__ int order[kMaxKrylov];
    __shared__ int dupc[kMaxKrylov];
    const int tid = threadIdx.x;

    // ---- load H_p (Hessenberg part only), Z = I --------------------------------
    for (int e = tid; e < p * p; e += kHT) {
        int r = e / p, c = e % p;
        Tl[e] = (r <= c + 1) ? H[r + (size_t)ldh * c] : cmk<double2>(0.0, 0.0);
        Z[c * p + r] = cmk<double2>(r == c ? 1.0 : 0.0, 0.0);
    }
    if (tid == 0) { sh_ihi = p - 1; sh_fail = 0; sh_iters = 0; }
    __syncthreads();

    // ---- shifted QR iteration ----------------------------------------------------
    int its = 0;           // iterations on the current eigenvalue (uniform)
    const int itmax = 30 * (p > 10 ? p : 10);
    while (true) {
        if (tid == 0) {
            int ihi = sh_ihi;
            int l = ihi;
            // deflation scan
            while (l > 0) {
                double2 sub = Tl[l * p + (l - 1)];
                double tst = cabs1(Tl[(l - 1) * p + (l - 1)]) + cabs1(Tl[l * p + l]);
                if (tst == 0.0) tst = 1.0;
                if (cabs1(sub) <= kEps * tst) { Tl[l * p + (l - 1)] = cmk<double2>(0.0, 0.0); break; }
                --l;
            }
            sh_l = l;
            if (l < ihi) {
                // shift
                double2 a = Tl[(ihi - 1) * p + (ihi - 1)], b = Tl[(ihi - 1) * p + ihi];
                double2 c2 = Tl[ihi * p + (ihi - 1)], d = Tl[ihi * p + ihi];
                double2 sft;
                if ((its + 1) % 10 == 0) {
                    // exceptional shift
                    double ex = 0.75 * fabs(c2.x) + fabs(d.x);
                    sft = cmk<double2>(d.x + ex, d.y);
                } else {
                    double2 half = cscale(csub(a, d), 0.5);
                    double2 disc = csqrt(cadd(cmul(half, half), cmul(b, c2)));
                    double2 mid = cscale(cadd(a, d), 0.5);
                    double2 l1 = cadd(mid, disc), l2 = csub(mid, disc);
                    sft = (cabs(csub(l1, d)) <= cabs(csub(l2, d))) ? l1 : l2;
                }
                sh_shift = sft;
                double2 x = csub(Tl[l * p + l], sft);
                double2 y = Tl[(l + 1) * p + l];
                double c;
                double2 s;
                givens(x, y, c, s);
                sh_c = c;
                sh_s = s;
            }
            sh_iters = sh_iters + (l < ihi ? 1 : 0);
        }
        __syncthreads();
        const int ihi = sh_ihi, l = sh_l;
        if (ihi <= 0) break;
        if (l == ihi) {  // eigenvalue T[ihi][ihi] converged
            __syncthreads();
            if (tid == 0) sh_ihi = ihi - 1;
            its = 0;
            __syncthreads();
            continue;
        }
        if (sh_iters > itmax) {
            if (tid == 0) sh_fail = 1;
            __syncthreads();
            break;
        }
        ++its;
        // bulge chase k = l .. ihi-1
        for (int kk = l; kk < ihi; ++kk) {
            if (kk > l) {
                if (tid == 0) {
                    double c;
                    double2 s;
                    givens(Tl[kk * p + (kk - 1)], Tl[(kk + 1) * p + (kk - 1)], c, s);
                    sh_c = c;
                    sh_s = s;
                }
                __syncthreads();
            }
            const double c = sh_c;
            const double2 s = sh_s;
            const double2 sc = cconj(s);
            // rows kk, kk+1: T <- G T on columns [max(kk-1, l), p)
            const int c0 = kk > l ? kk - 1 : l;
            for (int col = c0 + tid; col < p; col += kHT) {
                double2 a = Tl[kk * p + col], b = Tl[(kk + 1) * p + col];
                Tl[kk * p + col] = cadd(cscale(a, c), cmul(s, b));
                Tl[(kk + 1) * p + col] = csub(cscale(b, c), cmul(sc, a));
            }
            __syncthreads();
            if (kk > l && tid == 0) Tl[(kk + 1) * p + (kk - 1)] = cmk<double2>(0.0, 0.0);
            // columns kk, kk+1: T <- T G^H on rows [0, min(kk+2, ihi)], Z <- Z G^H
            const int r1 = (kk + 2 < ihi ? kk + 2 : ihi);
            for (int row = tid; row <= r1; row += kHT) {
                double2 a = Tl[row * p + kk], b = Tl[row * p + kk + 1];
                Tl[row * p + kk] = cadd(cscale(a, c), cmul(sc, b));
                Tl[row * p + kk + 1] = csub(cscale(b, c), cmul(s, a));
            }
            for (int row = tid; row < p; row += kHT) {
                double2 a = Z[kk * p + row], b = Z[(kk + 1) * p + row];
                Z[kk * p + row] = cadd(cscale(a, c), cmul(sc, b));
                Z[(kk + 1) * p + row] = csub(cscale(b, c), cmul(s, a));
            }
            __syncthreads();
        }
    }
    const int failed = sh_fail;

    // ---- eigenvalues ----------------------------------------------------------------
    for (int i = tid; i < p; i += kHT) mu[i] = Tl[i * p + i];

    // ---- eigenvectors of T: column sweep, S[i*p + r] holds the partial sums of
    //      vector i, the solution is written back into S.
    for (int e = tid; e < p * p; e += kHT) {
        int i = e / p, r = e % p;
        S[e] = (r < i) ? Tl[r * p + i] : cmk<double2>(r == i ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int c = p - 1; c >= 1; --c) {
        // finalise component c of every vector i > c
        for (int i = c + 1 + tid; i < p; i += kHT) {
            double2 lam = Tl[i * p + i];
            double2 den = csub(Tl[c * p + c], lam);
            double smin = kEps * cabs1(lam);
            if (smin < 1e-290) smin = 1e-290;
            if (cabs1(den) < smin) den = cmk<double2>(smin, 0.0);
            double2 z = cdiv(cmk<double2>(-S[i * p + c].x, -S[i * p + c].y), den);
            S[i * p + c] = z;
        }
        __syncthreads();
        // accumulate T[r][c] * z_i[c] into rows r < c of every vector i > c
        const int ni = p - 1 - c;  // vectors i = c+1 .. p-1
        for (int e = tid; e < ni * c; e += kHT) {
            int i = c + 1 + e / c, r = e % c;
            S[i * p + r] = cadd(S[i * p + r], cmul(Tl[r * p + c], S[i * p + c]));
        }
        __syncthreads();
    }
    // component 0 of every vector i >= 1
    for (int i = 1 + tid; i < p; i += kHT) {
        double2 lam = Tl[i * p + i];
        double2 den = csub(Tl[0], lam);
        double smin = kEps * cabs1(lam);
        if (smin < 1e-290) smin = 1e-290;
        if (cabs1(den) < smin) den = cmk<double2>(smin, 0.0);
        S[i * p] = cdiv(cmk<double2>(-S[i * p].x, -S[i * p].y), den);
    }
    __syncthreads();

    // ---- Y = Z z (z_i upper: components 0..i) -------------------------------------------
    for (int e = tid; e < p * p; e += kHT) {
        int i = e / p, r = e % p;
        double2 acc = cmk<double2>(0.0, 0.0);
        for (int c = 0; c <= i; ++c) acc = cadd(acc, cmul(Z[c * p + r], S[i * p + c]));
        Y[e] = acc;
    }
    __syncthreads();
    const double beta = beta_dev ? beta_dev[0] : beta_val;
    for (int i = tid; i < p; i += kHT) {
        double nrm = 0.0;
        for (int r = 0; r < p; ++r) nrm += cabs2(Y[i * p + r]);
        nrm = sqrt(nrm);
        double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int r = 0; r < p; ++r) Y[i * p + r] = cscale(Y[i * p + r], inv);
        res[i] = fabs(beta) * cabs(Y[i * p + (p - 1)]);
    }
    __syncthreads();
    if (sel == nullptr) {
        if (tid == 0 && rr) { rr->eig_fail = failed; rr->iters = sh_iters; }
        return;
    }

    // ---- wanted set ----------------------------------------------------------------------
    // rank by (-|mu|, -arg(mu)), ties by index
    for (int i = tid; i < p; i += kHT) {
        double mi = cabs(mu[i]), ai = atan2(mu[i].y, mu[i].x);
        int rank = 0;
        for (int j = 0; j < p; ++j) {
            if (j == i) continue;
            double mj = cabs(mu[j]), aj = atan2(mu[j].y, mu[j].x);
            bool before = (mj > mi) || (mj == mi && (aj > ai || (aj == ai && j < i)));
            rank += before ? 1 : 0;
        }
        order[rank] = i;
        // an unconverged value within its residual of some converged value
        int d = 0;
        if (!(res[i] <= tol)) {
            for (int j = 0; j < p; ++j)
                if (j != i && res[j] <= tol && cabs(csub(mu[i], mu[j])) <= res[i]) d = 1;
        }
        dupc[i] = d;
    }
    __syncthreads();
    if (tid == 0) {
        int nsel = 0, nconv = 0;
        for (int t = 0; t < p && nsel < k; ++t) {
            int i = order[t];
            bool conv = res[i] <= tol;
            bool take = conv;
            if (!conv) {
                take = !dupc[i];
                for (int a = 0; a < nsel && take; ++a)
                    if (cabs(csub(mu[i], mu[sel[a]])) <= res[i]) take = false;
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
        rr->iters = sh_iters;
        (void)T;
    }
}

}  // namespace

tsk_status hess_ritz_launch(const double2* H, int ldh, int p, const double* beta_dev, double beta_val,
                            double2* Z, double2* S, double2* mu, double2* Y, double* res, int k, double tol,
                            double T, int* sel, RitzResult* rr, hipStream_t s) {
    if (p < 1 || p > kMaxKrylov) return fail(TSK_EINVAL, "Hessenberg size must be in [1, 96]");
    size_t lds = size_t(p) * p * sizeof(double2);
    static bool attr_set = false;
    if (!attr_set) {
        TSK_HIP(hipFuncSetAttribute((const void*)k_hess_ritz, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(kMaxKrylov * kMaxKrylov * sizeof(double2))));
        attr_set = true;
    }
    hipLaunchKernelGGL(k_hess_ritz, dim3(1), dim3(kHT), lds, s, H, ldh, p, beta_dev, beta_val, Z, S, mu, Y,
                       res, k, tol, T, sel, rr);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

}  // namespace tsk
