// Kernels declared in krylov.hpp.
#include "krylov.hpp"

namespace tsk {

namespace {

// ---- element traits --------------------------------------------------------------
template <typename TS> struct ET;
template <> struct ET<double> {
    using A = double;  // FP64 working type
    static __device__ inline A acc(double v) { return v; }
    static __device__ inline double store(A v) { return v; }
};
template <> struct ET<float> {
    using A = double;
    static __device__ inline A acc(float v) { return double(v); }
    static __device__ inline float store(A v) { return float(v); }
};
template <> struct ET<double2> {
    using A = double2;
    static __device__ inline A acc(double2 v) { return v; }
    static __device__ inline double2 store(A v) { return v; }
};

__device__ inline double2 dotc(double v, double w) { return cmk<double2>(v * w, 0.0); }
__device__ inline double2 dotc(float v, double w) { return cmk<double2>(double(v) * w, 0.0); }
__device__ inline double2 dotc(double2 v, double2 w) { return cmulc(v, w); }
__device__ inline double nrm2(double w) { return w * w; }
__device__ inline double nrm2(double2 w) { return cabs2(w); }
// w - v h
__device__ inline double axmy(double w, double v, double2 h) { return w - v * h.x; }
__device__ inline double axmy(double w, float v, double2 h) { return w - double(v) * h.x; }
__device__ inline double2 axmy(double2 w, double2 v, double2 h) { return csub(w, cmul(v, h)); }
template <typename A> __device__ inline A zero_of();
template <> __device__ inline double zero_of<double>() { return 0.0; }
template <> __device__ inline double2 zero_of<double2>() { return cmk<double2>(0.0, 0.0); }
__device__ inline double scale_by(double w, double s) { return w * s; }
__device__ inline double2 scale_by(double2 w, double s) { return cscale(w, s); }
__device__ inline bool finite_of(double v) { return isfinite(v); }
__device__ inline bool finite_of(float v) { return isfinite(v); }
__device__ inline bool finite_of(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < kBT / kWave; ++q) t += red[q];
    return t;
}

// Dots of the LDS-staged chunk wl with every basis vector (wave-parallel).
template <typename TS, typename A>
__device__ inline void chunk_dots(const TS* __restrict__ V, int64_t ldv, int p, const A* wl, int64_t base,
                                  int64_t n, double2* __restrict__ partial) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t lim = n - base;
    for (int i = wave; i < p; i += kBT / kWave) {
        const TS* vi = V + i * ldv + base;
        double2 a = cmk<double2>(0.0, 0.0);
#pragma unroll 4
        for (int e = 0; e < kChunk / kWave; ++e) {
            int l = lane + e * kWave;
            if (l < lim) a = cadd(a, dotc(vi[l], wl[l]));
        }
        a = wave_sum(a);
        if (lane == 0) partial[size_t(blockIdx.x) * p + i] = a;
    }
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_dot(const TS* __restrict__ V, int64_t ldv, int p, const TS* __restrict__ w,
                                             int64_t n, double2* __restrict__ partial, double* __restrict__ pnrm) {
    using A = typename ET<TS>::A;
    __shared__ A wl[kChunk];
    __shared__ double red[kBT / kWave];
    const int64_t base = int64_t(blockIdx.x) * kChunk;
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
        int l = threadIdx.x + e * kBT;
        A x = (base + l < n) ? ET<TS>::acc(w[base + l]) : zero_of<A>();
        wl[l] = x;
        s2 += nrm2(x);
    }
    double t = block_sum(s2, red);
    if (threadIdx.x == 0) pnrm[blockIdx.x] = t;
    __syncthreads();
    chunk_dots(V, ldv, p, wl, base, n, partial);
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_update(const TS* __restrict__ V, int64_t ldv, int p,
                                                const double2* __restrict__ h, const TS* __restrict__ w_in,
                                                const typename ET<TS>::A* w64_in,  // may equal w64_out
                                                typename ET<TS>::A* w64_out, int64_t n, int dot,
                                                double2* __restrict__ partial, double* __restrict__ pnrm) {
    using A = typename ET<TS>::A;
    __shared__ A wl[kChunk];
    __shared__ double2 hl[kMaxKrylov + 1];
    __shared__ double red[kBT / kWave];
    for (int i = threadIdx.x; i < p; i += kBT) hl[i] = h[i];
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kChunk;
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
        int l = threadIdx.x + e * kBT;
        int64_t g = base + l;
        A x = zero_of<A>();
        if (g < n) {
            x = w64_in ? w64_in[g] : ET<TS>::acc(w_in[g]);
            for (int i = 0; i < p; ++i) x = axmy(x, V[i * ldv + g], hl[i]);
            w64_out[g] = x;
        }
        wl[l] = x;
        s2 += nrm2(x);
    }
    double t = block_sum(s2, red);
    if (threadIdx.x == 0) pnrm[blockIdx.x] = t;
    if (dot) {
        __syncthreads();
        chunk_dots(V, ldv, p, wl, base, n, partial);
    }
}

__global__ void k_reduce(const double2* __restrict__ partial, int nblk, int p, double2* __restrict__ h,
                         double2* __restrict__ Hcol, int first, const double* __restrict__ pnrm,
                         double* __restrict__ scal, int slot) {
    for (int i = threadIdx.x; i < p; i += blockDim.x) {
        double2 s = cmk<double2>(0.0, 0.0);
        for (int b = 0; b < nblk; ++b) s = cadd(s, partial[size_t(b) * p + i]);
        h[i] = s;
        if (Hcol) Hcol[i] = first ? s : cadd(Hcol[i], s);
    }
    if (pnrm && threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += pnrm[b];
        scal[slot] = s;
    }
}

__global__ void k_finalize(const double* __restrict__ pnrm, int nblk, const double* __restrict__ scal, int win_slot,
                           double2* __restrict__ Hsub, double* __restrict__ beta_out, RitzResult* __restrict__ rr) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += pnrm[b];
    double beta = sqrt(s);
    double win = sqrt(scal[win_slot]);
    *Hsub = cmk<double2>(beta, 0.0);
    *beta_out = beta;
    rr->beta = beta;
    rr->w_in = win;
    rr->nonfinite = !(isfinite(beta) && isfinite(win));
    rr->breakdown = (beta <= 64.0 * 2.220446049250313e-16 * win) ? 1 : 0;
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_scale(const typename ET<TS>::A* __restrict__ w64,
                                               const double* __restrict__ beta, TS* __restrict__ v, int64_t n) {
    const double b = beta[0];
    const double inv = (b > 0.0 && isfinite(b)) ? 1.0 / b : 0.0;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
        v[g] = ET<TS>::store(scale_by(w64[g], inv));
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_scale_state(const TS* __restrict__ x, const double* __restrict__ scal,
                                                     int slot, TS* __restrict__ v, int64_t n) {
    const double s2 = scal[slot];
    const double inv = (s2 > 0.0 && isfinite(s2)) ? 1.0 / sqrt(s2) : 0.0;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
        v[g] = ET<TS>::store(scale_by(ET<TS>::acc(x[g]), inv));
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_ritz(const TS* __restrict__ V, int64_t ldv, int p,
                                              const double2* __restrict__ Y, const int* __restrict__ sel, int k,
                                              double2* __restrict__ X, int64_t n) {
    const int s = blockIdx.y;
    const double2* y = Y + size_t(s) * p;  // unit Ritz coordinates of wanted pair s
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x) {
        double2 acc = cmk<double2>(0.0, 0.0);
        for (int i = 0; i < p; ++i) {
            typename ET<TS>::A v = ET<TS>::acc(V[i * ldv + g]);
            if constexpr (sizeof(v) == sizeof(double)) acc = cadd(acc, cscale(y[i], double(v)));
            else acc = cadd(acc, cmul(y[i], v));
        }
        X[size_t(s) * n + g] = acc;
    }
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_check_finite(const TS* __restrict__ x, int64_t n, int* __restrict__ flag) {
    int bad = 0;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
        bad |= finite_of(x[g]) ? 0 : 1;
    if (bad) atomicOr(flag, 1);
}

inline int grid_for(int64_t n) {
    int64_t b = (n + kBT - 1) / kBT;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return int(b);
}

}  // namespace

template <typename TS>
void launch_dot(const TS* V, int64_t ldv, int p, const TS* w, int64_t n, double2* partial, double* pnrm,
                hipStream_t s) {
    hipLaunchKernelGGL(k_dot<TS>, dim3(cgs_blocks(n)), dim3(kBT), 0, s, V, ldv, p, w, n, partial, pnrm);
}

void launch_reduce(const double2* partial, int nblk, int p, double2* h, double2* Hcol, int first,
                   const double* pnrm, double* scal, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(128), 0, s, partial, nblk, p, h, Hcol, first, pnrm, scal, slot);
}

template <typename TS>
void launch_update(const TS* V, int64_t ldv, int p, const double2* h, const TS* w_in, const void* w64_in,
                   void* w64_out, int64_t n, bool dot, double2* partial, double* pnrm, hipStream_t s) {
    using A = typename ET<TS>::A;
    hipLaunchKernelGGL(k_update<TS>, dim3(cgs_blocks(n)), dim3(kBT), 0, s, V, ldv, p, h, w_in,
                       static_cast<const A*>(w64_in), static_cast<A*>(w64_out), n, dot ? 1 : 0, partial, pnrm);
}

void launch_finalize(const double* pnrm, int nblk, const double* scal, int win_slot, double2* Hsub,
                     double* beta_out, RitzResult* rr, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, pnrm, nblk, scal, win_slot, Hsub, beta_out, rr);
}

template <typename TS>
void launch_scale(const void* w64, const double* beta, TS* v, int64_t n, hipStream_t s) {
    using A = typename ET<TS>::A;
    hipLaunchKernelGGL(k_scale<TS>, dim3(grid_for(n)), dim3(kBT), 0, s, static_cast<const A*>(w64), beta, v, n);
}

template <typename TS>
void launch_scale_state(const TS* x, const double* scal, int slot, TS* v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_state<TS>, dim3(grid_for(n)), dim3(kBT), 0, s, x, scal, slot, v, n);
}

template <typename TS>
void launch_ritz_vectors(const TS* V, int64_t ldv, int p, const double2* Y, const int* sel, int k, double2* X,
                         int64_t n, hipStream_t s) {
    int gx = grid_for(n);
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_ritz<TS>, dim3(gx, k), dim3(kBT), 0, s, V, ldv, p, Y, sel, k, X, n);
}

template <typename TS>
void launch_check_finite(const TS* x, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite<TS>, dim3(grid_for(n)), dim3(kBT), 0, s, x, n, flag);
}

#define TSK_INST(TS)                                                                                              \
    template void launch_dot<TS>(const TS*, int64_t, int, const TS*, int64_t, double2*, double*, hipStream_t);    \
    template void launch_update<TS>(const TS*, int64_t, int, const double2*, const TS*, const void*, void*,       \
                                    int64_t, bool, double2*, double*, hipStream_t);                               \
    template void launch_scale<TS>(const void*, const double*, TS*, int64_t, hipStream_t);                       \
    template void launch_scale_state<TS>(const TS*, const double*, int, TS*, int64_t, hipStream_t);              \
    template void launch_ritz_vectors<TS>(const TS*, int64_t, int, const double2*, const int*, int, double2*,    \
                                          int64_t, hipStream_t);                                                  \
    template void launch_check_finite<TS>(const TS*, int64_t, int*, hipStream_t);
TSK_INST(double)
TSK_INST(float)
TSK_INST(double2)
#undef TSK_INST

}  // namespace tsk
