// Fixed-point solvers on the nonlinear time-stepper (Sec. 3.1): selective
// frequency damping, the recursive projection method and BoostConv.  The
// solvers are host loops around device work: the nonlinear steps of the
// Navier-Stokes operator (kolmo2d.hip, ROW_NL pipeline) and the small vector
// kernels below.  Per iteration only the residual norm crosses to the host.
//
// SFD (Sec. 3.1.1): the extended system X' = F(X) - chi (X - Y), Y' = (X - Y)/Delta
// by Strang splitting: the coupling is linear with B = [[-chi, chi], [1/Delta,
// -1/Delta]] and B^2 = -s B, s = chi + 1/Delta, so exp(t B) = I + (1 - e^{-s t})/s B
// exactly; a step is half the coupling, one nonlinear step, half the coupling.
// RPM (Sec. 3.1.2): U and H = U^T M U come from an Arnoldi factorisation of the
// Jacobian about the initial iterate (the operator's base flow set to it,
// started from the initial residual) contracted by the Krylov-Schur kernel
// (kept set |mu| >= 1 - delta); then x~ <- x + U ((I - H)^-1 z - z), z = U^T r,
// r = G(x~) - x~, x = G(x~).  BoostConv (Sec. 3.1.3): the corrections xi_j and
// residual decrements y_j = r_j - r_{j+1} of the last m iterations,
// c = (Y^T Y)^-1 Y^T r, xi = r + (X - Y) c, x~ <- x~ + xi.
// Dot products are FP64, reduced in a fixed order (bitwise reproducible).
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

constexpr int kFT = 256;        // threads of the vector kernels
constexpr int kFChunk = 4096;   // elements per partial sum

inline int fblocks(int64_t n) { return int((n + kFChunk - 1) / kFChunk); }

template <typename TS> __device__ inline double rd(const TS* p, int64_t i) { return double(p[i]); }

__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kFT / 64; ++q) t += red[q];
    __syncthreads();
    return t;
}

// partial[(j * nb) + b] = sum over chunk b of A_j[e] * B_i[e] for the pair list:
// vectors A_j = A + j * lda (j < na) against vector r, or the pair (j, i) of Y
// when gram.  Grid (nb, npairs).
template <typename TS>
__global__ __launch_bounds__(kFT) void k_pdot(const TS* __restrict__ A, int64_t lda, const TS* __restrict__ r,
                                              int64_t n, double* __restrict__ partial, int nb) {
    __shared__ double red[kFT / 64];
    const int b = blockIdx.x, j = blockIdx.y;
    const TS* a = A + j * lda;
    const int64_t e0 = int64_t(b) * kFChunk, e1 = e0 + kFChunk < n ? e0 + kFChunk : n;
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kFT) s += rd(a, e) * rd(r, e);
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[size_t(j) * nb + b] = s;
}

// out[j] = sum_b partial[j * nb + b] (fixed order), one thread per output.
__global__ void k_psum(const double* __restrict__ partial, int nb, int count, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[size_t(j) * nb + b];
    out[j] = s;
}

// r = xn - x and partial sums of r^2.
template <typename TS>
__global__ __launch_bounds__(kFT) void k_resid(const TS* __restrict__ xn, const TS* __restrict__ x,
                                               TS* __restrict__ r, int64_t n, double* __restrict__ partial) {
    __shared__ double red[kFT / 64];
    const int b = blockIdx.x;
    const int64_t e0 = int64_t(b) * kFChunk, e1 = e0 + kFChunk < n ? e0 + kFChunk : n;
    double s = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kFT) {
        const double d = rd(xn, e) - rd(x, e);
        r[e] = TS(d);
        s += d * d;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[b] = s;
}

// (X, Y) <- E (Xin, Y) elementwise, E a 2 x 2 matrix; Xin may alias X.
template <typename TS>
__global__ void k_couple(TS* X, TS* __restrict__ Y, const TS* Xin, int64_t n, double e00, double e01, double e10,
                         double e11) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        const double a = rd(Xin, e), y = rd(Y, e);
        X[e] = TS(e00 * a + e01 * y);
        Y[e] = TS(e10 * a + e11 * y);
    }
}

// out = base + sum_j c_j (P_j - Q_j) (Q null: sum_j c_j P_j); out may alias base.
template <typename TS>
__global__ void k_combine(TS* out, const TS* base, const TS* __restrict__ P, const TS* __restrict__ Q, int64_t ld,
                          const double* __restrict__ c, int np, int64_t n) {
    __shared__ double cs[kMaxKrylov];
    for (int j = threadIdx.x; j < np; j += blockDim.x) cs[j] = c[j];
    __syncthreads();
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        double v = rd(base, e);
        for (int j = 0; j < np; ++j) v += cs[j] * (rd(P, j * ld + e) - (Q ? rd(Q, j * ld + e) : 0.0));
        out[e] = TS(v);
    }
}

// out = a x + b y elementwise (out may alias x or y).
template <typename TS>
__global__ void k_lincomb(TS* out, double a, const TS* x, double b, const TS* y, int64_t n) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
        out[e] = TS(a * rd(x, e) + b * rd(y, e));
}

// Dense solve A c = z (p x p, column-major with leading dimension lda) by Gaussian
// elimination with partial pivoting on one wavefront (lane 0 chooses the pivot,
// the lanes update the rows).  mode 0: A = I - H (RPM), out = c - z; mode 1:
// A = G (BoostConv normal equations), out = c.  A pivot below eps * max|A|
// is replaced by that floor.
__global__ __launch_bounds__(64) void k_small_solve(const double* __restrict__ Ain, int lda, const double* __restrict__ z,
                                                    int p, int mode, double* __restrict__ out) {
    __shared__ double A[kMaxKrylov][kMaxKrylov + 1];
    __shared__ double b[kMaxKrylov];
    __shared__ int piv;
    __shared__ double amax;
    const int lane = threadIdx.x;
    for (int e = lane; e < p * p; e += 64) {
        const int r = e % p, c = e / p;
        const double a = Ain[r + size_t(lda) * c];
        A[r][c] = mode == 0 ? (r == c ? 1.0 : 0.0) - a : a;
    }
    for (int r = lane; r < p; r += 64) b[r] = z[r];
    __syncthreads();
    if (lane == 0) {
        double m = 0.0;
        for (int r = 0; r < p; ++r)
            for (int c = 0; c < p; ++c) m = fmax(m, fabs(A[r][c]));
        amax = m > 0.0 ? m : 1.0;
    }
    __syncthreads();
    const double floor_ = 2.220446049250313e-16 * amax;
    for (int k = 0; k < p; ++k) {
        if (lane == 0) {
            int q = k;
            for (int r = k + 1; r < p; ++r)
                if (fabs(A[r][k]) > fabs(A[q][k])) q = r;
            piv = q;
        }
        __syncthreads();
        const int q = piv;
        if (q != k) {
            for (int c = lane; c < p; c += 64) {
                const double t = A[k][c];
                A[k][c] = A[q][c];
                A[q][c] = t;
            }
            if (lane == 0) {
                const double t = b[k];
                b[k] = b[q];
                b[q] = t;
            }
        }
        __syncthreads();
        if (lane == 0 && fabs(A[k][k]) < floor_) A[k][k] = A[k][k] < 0.0 ? -floor_ : floor_;
        __syncthreads();
        for (int r = k + 1 + lane; r < p; r += 64) {
            const double f = A[r][k] / A[k][k];
            for (int c = k; c < p; ++c) A[r][c] -= f * A[k][c];
            b[r] -= f * b[k];
        }
        __syncthreads();
    }
    if (lane == 0) {
        for (int r = p - 1; r >= 0; --r) {
            double v = b[r];
            for (int c = r + 1; c < p; ++c) v -= A[r][c] * b[c];
            b[r] = v / A[r][r];
        }
        for (int r = 0; r < p; ++r) out[r] = mode == 0 ? b[r] - z[r] : b[r];
    }
}

inline int egrid(int64_t n) {
    int64_t b = (n + 255) / 256;
    return int(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

// Device scratch of one solver run and its residual read-back.
struct FpWork {
    DevBuf partial, sums, small;
    double* host = nullptr;  // pinned: residual^2
    ~FpWork() {
        if (host) (void)hipHostFree(host);
    }
    tsk_status init(int64_t n, int nvec) {
        TSK_TRY(partial.ensure(size_t(fblocks(n)) * (nvec + 1) * (nvec + 1) * sizeof(double)));
        TSK_TRY(sums.ensure(size_t(nvec + 1) * (nvec + 1) * sizeof(double)));
        TSK_TRY(small.ensure(size_t(2 * kMaxKrylov) * sizeof(double)));
        TSK_HIP(hipHostMalloc((void**)&host, 8 * sizeof(double), 0));
        return TSK_OK;
    }
};

// r = xn - x; returns ||r|| (synchronises the stream).
template <typename TS>
tsk_status residual(const TS* xn, const TS* x, TS* r, int64_t n, FpWork& fw, hipStream_t s, double* norm) {
    const int nb = fblocks(n);
    hipLaunchKernelGGL(k_resid<TS>, dim3(nb), dim3(kFT), 0, s, xn, x, r, n, fw.partial.as<double>());
    hipLaunchKernelGGL(k_psum, dim3(1), dim3(64), 0, s, fw.partial.as<double>(), nb, 1, fw.sums.as<double>());
    TSK_HIP(hipMemcpyAsync(fw.host, fw.sums.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    *norm = std::sqrt(fw.host[0]);
    return TSK_OK;
}

// out[j] = A_j . r for j < na (A_j = A + j * lda).
template <typename TS>
void dots(const TS* A, int64_t lda, int na, const TS* r, int64_t n, FpWork& fw, double* out, hipStream_t s) {
    const int nb = fblocks(n);
    hipLaunchKernelGGL(k_pdot<TS>, dim3(nb, na), dim3(kFT), 0, s, A, lda, r, n, fw.partial.as<double>(), nb);
    hipLaunchKernelGGL(k_psum, dim3((na + 63) / 64), dim3(64), 0, s, fw.partial.as<double>(), nb, na, out);
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

void fill_info(tsk_fp_info* info, int status, int iters, int64_t steps, int basis, double res, double ms) {
    if (!info) return;
    info->status = status;
    info->iterations = iters;
    info->time_steps = steps;
    info->basis_dim = basis;
    info->residual = res;
    info->ms_total = ms;
}

// ---- selective frequency damping --------------------------------------------------------
template <typename TS>
tsk_status sfd_t(Operator* op, void* xv, double chi, double delta, int check_every, double tol, int max_checks,
                 double* hist, tsk_fp_info* info) {
    Timer tm;
    const hipStream_t s = op->stream;
    const int64_t n = op->n;
    const double h = kolmo_dt(op);
    TS* X = static_cast<TS*>(xv);
    DevBuf Yb, Xs, R;
    TSK_TRY(Yb.ensure(op->state_bytes()));
    TSK_TRY(Xs.ensure(op->state_bytes()));
    TSK_TRY(R.ensure(op->state_bytes()));
    FpWork fw;
    TSK_TRY(fw.init(n, 1));
    TS* Y = Yb.as<TS>();
    TSK_HIP(hipMemcpyAsync(Y, X, op->state_bytes(), hipMemcpyDeviceToDevice, s));
    // exp(h/2 B) = I + (1 - e^{-s h/2})/s B, B = [[-chi, chi], [1/Delta, -1/Delta]]
    const double sr = chi + 1.0 / delta, g = (1.0 - std::exp(-sr * 0.5 * h)) / sr;
    const double e00 = 1.0 - g * chi, e01 = g * chi, e10 = g / delta, e11 = 1.0 - g / delta;
    const int eg = egrid(n);
    double res = INFINITY;
    int checks = 0;
    int64_t steps = 0;
    int status = TSK_NOT_CONVERGED;
    for (; checks < max_checks;) {
        for (int q = 0; q < check_every; ++q) {
            hipLaunchKernelGGL(k_couple<TS>, dim3(eg), dim3(256), 0, s, X, Y, X, n, e00, e01, e10, e11);
            TSK_TRY(kolmo_nonlinear_step(op, X, Xs.ptr, 1));
            hipLaunchKernelGGL(k_couple<TS>, dim3(eg), dim3(256), 0, s, X, Y, Xs.as<TS>(), n, e00, e01, e10, e11);
        }
        steps += check_every;
        TSK_TRY(kolmo_nonlinear_step(op, X, Xs.ptr, 1));
        double nr;
        TSK_TRY(residual<TS>(Xs.as<TS>(), X, R.as<TS>(), n, fw, s, &nr));
        res = nr / h;
        if (hist) hist[checks] = res;
        ++checks;
        if (!std::isfinite(res)) return fail(TSK_ENONFINITE, "SFD iterate is not finite");
        if (res <= tol) {
            status = TSK_OK;
            break;
        }
    }
    if (status == TSK_OK) TSK_TRY(kolmo_base_from_state(op, X));
    fill_info(info, status, checks, steps, 0, res, tm.ms());
    return tsk_status(status);
}

// ---- recursive projection method ---------------------------------------------------------
template <typename TS>
tsk_status rpm_t(Operator* op, void* xv, int m, int k, double delta, double tol, int max_iter, double* hist,
                 tsk_fp_info* info) {
    Timer tm;
    const hipStream_t s = op->stream;
    const int64_t n = op->n;
    TS* x = static_cast<TS*>(xv);
    const size_t sb = op->state_bytes();
    DevBuf xn, r;
    TSK_TRY(xn.ensure(sb));
    TSK_TRY(r.ensure(sb));
    FpWork fw;
    TSK_TRY(fw.init(n, m));
    // initial residual: the Arnoldi start vector
    TSK_TRY(kolmo_nonlinear_step(op, x, xn.ptr, 0));
    double nr0;
    TSK_TRY(residual<TS>(xn.as<TS>(), x, r.as<TS>(), n, fw, s, &nr0));
    if (!std::isfinite(nr0)) return fail(TSK_ENONFINITE, "initial iterate is not finite");
    if (nr0 <= tol) {
        if (hist) hist[0] = nr0;
        TSK_TRY(kolmo_base_from_state(op, x));
        fill_info(info, TSK_OK, 0, 0, 0, nr0, tm.ms());
        return TSK_OK;
    }
    // Jacobian about the initial iterate, Arnoldi from r0, Krylov-Schur contraction
    TSK_TRY(kolmo_base_from_state(op, x));
    const void* v0 = r.ptr;
    uint64_t seed = 0;
    tsk_arnoldi_info ai{};
    const tsk_status ast = arnoldi_batch(&op, 1, m, 1, 0.0, &v0, &seed, nullptr, nullptr, nullptr, nullptr, &ai);
    if (ast < 0) return ast;
    ArnoldiWork& aw = op->aw;
    const int order = aw.steps;
    if (order < 3) return fail(TSK_BREAKDOWN, "the Jacobian's Krylov space has dimension < 3");
    DevBuf Hr, mu, resv, Hn, W, U;
    TSK_TRY(Hr.ensure(size_t(m + 1) * m * sizeof(double)));
    TSK_TRY(mu.ensure(size_t(m) * sizeof(double2)));
    TSK_TRY(resv.ensure(size_t(m) * sizeof(double)));
    TSK_TRY(Hn.ensure(size_t(order + 1) * order * sizeof(double)));
    TSK_TRY(W.ensure(size_t(order) * order * sizeof(double)));
    // real parts of H ((m+1) x m complex, ld m+1)
    TSK_HIP(hipMemcpy2DAsync(Hr.ptr, sizeof(double), aw.H.ptr, sizeof(double2), sizeof(double), size_t(m + 1) * m,
                             hipMemcpyDeviceToDevice, s));
    double beta = 0.0;
    TSK_HIP(hipMemcpyAsync(&beta, Hr.as<double>() + order + size_t(m + 1) * (order - 1), sizeof(double),
                           hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    int kp = 0;
    double bnew = 0.0;
    TSK_TRY(ks_contract_standalone(Hr.as<double>(), m + 1, order, beta, std::min(k, order - 2), delta, order - 2,
                                   mu.ptr, resv.as<double>(), Hn.as<double>(), W.as<double>(), &kp, &bnew, s));
    TSK_TRY(U.ensure(size_t(kp + 1) * aw.ldv * sizeof(TS)));
    launch_rotate<TS>(aw.Vcur, U.ptr, W.as<double>(), n, aw.ldv, order, kp, s);
    // iterations
    double* z = fw.small.as<double>();
    double* d = z + kMaxKrylov;
    double res = nr0;
    int it = 0, status = TSK_NOT_CONVERGED;
    const int eg = egrid(n);
    for (; it < max_iter; ++it) {
        if (it > 0) {
            TSK_TRY(kolmo_nonlinear_step(op, x, xn.ptr, 0));
            TSK_TRY(residual<TS>(xn.as<TS>(), x, r.as<TS>(), n, fw, s, &res));
        }
        if (hist) hist[it] = res;
        if (!std::isfinite(res)) return fail(TSK_ENONFINITE, "RPM iterate is not finite");
        if (res <= tol) {
            status = TSK_OK;
            break;
        }
        dots<TS>(U.as<TS>(), aw.ldv, kp, r.as<TS>(), n, fw, z, s);
        hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, s, Hn.as<double>(), order + 1, z, kp, 0, d);
        hipLaunchKernelGGL(k_combine<TS>, dim3(eg), dim3(256), 0, s, x, xn.as<TS>(), U.as<TS>(),
                           static_cast<const TS*>(nullptr), aw.ldv, d, kp, n);
        TSK_HIP(hipGetLastError());
    }
    if (status == TSK_OK) TSK_TRY(kolmo_base_from_state(op, x));
    fill_info(info, status, it, int64_t(it + 1) * kolmo_nsteps(op), kp, res, tm.ms());
    return tsk_status(status);
}

// ---- BoostConv -----------------------------------------------------------------------------
template <typename TS>
tsk_status boostconv_t(Operator* op, void* xv, int m, double tol, int max_iter, double* hist, tsk_fp_info* info) {
    Timer tm;
    const hipStream_t s = op->stream;
    const int64_t n = op->n;
    const int64_t ldv = (n + 63) / 64 * 64;
    TS* x = static_cast<TS*>(xv);
    const size_t sb = op->state_bytes();
    DevBuf xn, r, rp, xip, Xb, Yb, Gm;
    TSK_TRY(xn.ensure(sb));
    TSK_TRY(r.ensure(sb));
    TSK_TRY(rp.ensure(sb));
    TSK_TRY(xip.ensure(sb));
    TSK_TRY(Xb.ensure(size_t(m) * ldv * sizeof(TS)));
    TSK_TRY(Yb.ensure(size_t(m) * ldv * sizeof(TS)));
    TSK_TRY(Gm.ensure(size_t(m) * m * sizeof(double)));
    FpWork fw;
    TSK_TRY(fw.init(n, m));
    double* bvec = fw.small.as<double>();
    double* c = bvec + kMaxKrylov;
    const int eg = egrid(n);
    int it = 0, count = 0, status = TSK_NOT_CONVERGED;
    double res = INFINITY;
    for (; it < max_iter; ++it) {
        TSK_TRY(kolmo_nonlinear_step(op, x, xn.ptr, 0));
        TSK_TRY(residual<TS>(xn.as<TS>(), x, r.as<TS>(), n, fw, s, &res));
        if (hist) hist[it] = res;
        if (!std::isfinite(res)) return fail(TSK_ENONFINITE, "BoostConv iterate is not finite");
        if (res <= tol) {
            status = TSK_OK;
            break;
        }
        if (it > 0) {  // the newest pair (xi_{k-1}, r_{k-1} - r_k) replaces the oldest
            const int slot = count % m;
            hipLaunchKernelGGL(k_lincomb<TS>, dim3(eg), dim3(256), 0, s, Yb.as<TS>() + slot * ldv, 1.0, rp.as<TS>(),
                               -1.0, r.as<TS>(), n);
            TSK_HIP(hipMemcpyAsync(Xb.as<TS>() + slot * ldv, xip.ptr, sb, hipMemcpyDeviceToDevice, s));
            ++count;
        }
        const int nh = std::min(count, m);
        if (nh > 0) {
            // c = (Y^T Y)^-1 Y^T r, xi = r + sum_j c_j (X_j - Y_j)
            for (int j = 0; j < nh; ++j)
                dots<TS>(Yb.as<TS>(), ldv, nh, Yb.as<TS>() + j * ldv, n, fw, Gm.as<double>() + size_t(j) * nh, s);
            dots<TS>(Yb.as<TS>(), ldv, nh, r.as<TS>(), n, fw, bvec, s);
            hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, s, Gm.as<double>(), nh, bvec, nh, 1, c);
            hipLaunchKernelGGL(k_combine<TS>, dim3(eg), dim3(256), 0, s, xip.as<TS>(), r.as<TS>(), Xb.as<TS>(),
                               Yb.as<TS>(), ldv, c, nh, n);
        } else {
            TSK_HIP(hipMemcpyAsync(xip.ptr, r.ptr, sb, hipMemcpyDeviceToDevice, s));
        }
        hipLaunchKernelGGL(k_lincomb<TS>, dim3(eg), dim3(256), 0, s, x, 1.0, x, 1.0, xip.as<TS>(), n);
        TSK_HIP(hipMemcpyAsync(rp.ptr, r.ptr, sb, hipMemcpyDeviceToDevice, s));
        TSK_HIP(hipGetLastError());
    }
    if (status == TSK_OK) TSK_TRY(kolmo_base_from_state(op, x));
    fill_info(info, status, it, int64_t(it + 1) * kolmo_nsteps(op), std::min(count, m), res, tm.ms());
    return tsk_status(status);
}

tsk_status check_nl(Operator* op, void* x) {
    if (!op) return fail(TSK_EINVAL, "null operator");
    if (!is_kolmo(op)) return fail(TSK_EINVAL, "fixed-point solvers need a Navier-Stokes operator");
    if (!x) return fail(TSK_EINVAL, "null state");
    if (!op->params_set) return fail(TSK_ESTATE, "set Re, alpha, dt and T first");
    return TSK_OK;
}

}  // namespace

tsk_status fixed_point_sfd(Operator* op, void* x, double chi, double delta, int check_every, double tol,
                           int max_checks, double* hist, tsk_fp_info* info) {
    TSK_TRY(check_nl(op, x));
    if (!(chi > 0.0) || !(delta > 0.0) || !std::isfinite(chi) || !std::isfinite(delta))
        return fail(TSK_EINVAL, "chi and Delta must be positive and finite");
    if (check_every < 1 || max_checks < 1) return fail(TSK_EINVAL, "check_every and max_checks must be >= 1");
    if (!(tol >= 0.0)) return fail(TSK_EINVAL, "tol must be >= 0");
    if (op->kind == StateKind::Real32)
        return sfd_t<float>(op, x, chi, delta, check_every, tol, max_checks, hist, info);
    return sfd_t<double>(op, x, chi, delta, check_every, tol, max_checks, hist, info);
}

tsk_status fixed_point_rpm(Operator* op, void* x, int m, int k, double delta, double tol, int max_iter, double* hist,
                           tsk_fp_info* info) {
    TSK_TRY(check_nl(op, x));
    if (k < 1 || m < k + 2 || m > kMaxKrylov || int64_t(m) > op->n)
        return fail(TSK_EINVAL, "need 1 <= k, k + 2 <= m <= 96 and m <= state length");
    if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(TSK_EINVAL, "delta must be finite and >= 0");
    if (max_iter < 1 || !(tol >= 0.0)) return fail(TSK_EINVAL, "need max_iter >= 1 and tol >= 0");
    if (op->kind == StateKind::Real32) return rpm_t<float>(op, x, m, k, delta, tol, max_iter, hist, info);
    return rpm_t<double>(op, x, m, k, delta, tol, max_iter, hist, info);
}

tsk_status fixed_point_boostconv(Operator* op, void* x, int m, double tol, int max_iter, double* hist,
                                 tsk_fp_info* info) {
    TSK_TRY(check_nl(op, x));
    if (m < 1 || m > kMaxKrylov) return fail(TSK_EINVAL, "history length must be in [1, 96]");
    if (max_iter < 1 || !(tol >= 0.0)) return fail(TSK_EINVAL, "need max_iter >= 1 and tol >= 0");
    if (op->kind == StateKind::Real32) return boostconv_t<float>(op, x, m, tol, max_iter, hist, info);
    return boostconv_t<double>(op, x, m, tol, max_iter, hist, info);
}

}  // namespace tsk
