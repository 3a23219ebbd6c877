// Kernels declared in krylov.hpp.
#include <type_traits>

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
__device__ inline double2 cgain(double2 y, double v) { return cscale(y, v); }
__device__ inline double2 cgain(double2 y, double2 v) { return cmul(y, v); }

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

// Load through a global-address-space pointer: the compiler then emits
// global loads, which count only against the vector-memory counter, so waits
// for LDS traffic do not also wait for them (flat loads count against both).
template <typename T> __device__ inline T ldg(const T* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(1))) T*)p)[i];
#else
    return p[i];  // host pass only: device functions are never run on the host
#endif
}

// Dots of the LDS-staged chunk wl (kChunk elements) with every basis vector
// (wave-parallel).  Wave w takes the vectors i = w, w + 4, w + 8, ...; it loads
// kDotU of them at once, with clamped indices and no branches so that every
// load is in flight before the first wait, and accumulates each vector in the
// element order e = 0, 1, ... (elements beyond the state skipped) before its
// shuffle reduction.
constexpr int kDotU = 8;
template <typename TS, typename A>
__device__ inline void chunk_dots(const TS* __restrict__ V, int64_t ldv, int p, const A* wl, int64_t base,
                                  int64_t n, double2* __restrict__ partial) {
    constexpr bool kReal = !std::is_same<TS, double2>::value;  // real states: the dots are real
    // complex states load 4 vectors at a time (8 of them would not fit the registers)
    constexpr int NW = kBT / kWave, E = kChunk / kWave, U = kReal ? kDotU : 4;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t lim = n - base;  // >= 1
    A wv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) wv[e] = wl[lane + e * kWave];
    for (int i0 = wave; i0 < p; i0 += NW * U) {
        TS vv[U][E];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + NW * u;
            const TS* vi = V + int64_t(i < p ? i : p - 1) * ldv + base;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t l = lane + e * kWave;
                vv[u][e] = ldg(vi, l < lim ? l : lim - 1);
            }
        }
        double2 a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = cmk<double2>(0.0, 0.0);
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (lane + e * kWave < lim) a[u] = cadd(a[u], dotc(vv[u][e], wv[e]));
            if constexpr (kReal)
                a[u].x = wave_sum(a[u].x);  // the imaginary parts are exact zeros
            else
                a[u] = wave_sum(a[u]);
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + NW * u;
                if (i < p) {
                    if constexpr (kReal)  // real partials: half the bytes for every block to reduce
                        reinterpret_cast<double*>(partial)[size_t(blockIdx.x) * p + i] = a[u].x;
                    else
                        partial[size_t(blockIdx.x) * p + i] = a[u];
                }
            }
        }
    }
}

// x[e] - sum_i V[i][g_e] h_i for the thread's EPT elements g_e = g0 + e kBT,
// subtracted in the order i = 0, 1, ..., p-1; the loads of U = 16 basis vectors
// are issued together ahead of their products.  Elements beyond the state
// (g_e >= n) read element n - 1 instead and come back as garbage: the caller
// discards them.
template <int EPT, typename TS, typename A>
__device__ inline void project_out(A (&x)[EPT], const TS* __restrict__ V, int64_t ldv, int64_t g0, int64_t n,
                                   const double2* hl, int p) {
    constexpr int U = 16;
    int64_t g[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) g[e] = g0 + e * kBT < n ? g0 + e * kBT : n - 1;
    int i0 = 0;
    for (; i0 + U <= p; i0 += U) {
        TS vv[U][EPT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < EPT; ++e) vv[u][e] = ldg(V, int64_t(i0 + u) * ldv + g[e]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < EPT; ++e) x[e] = axmy(x[e], vv[u][e], hl[i0 + u]);
    }
    if (i0 < p) {
        // the remaining p - i0 < U vectors as one more batch (indices clamped to
        // p - 1 for the loads, the extra products skipped): same order, one
        // memory latency instead of one per vector
        TS vv[U][EPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u < p ? i0 + u : p - 1;
#pragma unroll
            for (int e = 0; e < EPT; ++e) vv[u][e] = ldg(V, int64_t(i) * ldv + g[e]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u < p)
#pragma unroll
                for (int e = 0; e < EPT; ++e) x[e] = axmy(x[e], vv[u][e], hl[i0 + u]);
    }
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_check_finite(const KryDesc* __restrict__ Dv) {
    const KryDesc& d = Dv[blockIdx.y];
    const TS* x = static_cast<const TS*>(d.x0);
    int bad = 0;
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < d.n; g += int64_t(gridDim.x) * blockDim.x)
        bad |= finite_of(x[g]) ? 0 : 1;
    if (bad) atomicOr(reinterpret_cast<int*>(d.scal + 32), 1);
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_dot(const KryDesc* __restrict__ Dv, int p, int from_x0) {
    using A = typename ET<TS>::A;
    const KryDesc& d = Dv[blockIdx.y];
    if (!d.active || int(blockIdx.x) >= d.nblk) return;
    if (!from_x0) {
        p += d.poff;  // the instance's own order (batched restart phase)
        if (p > d.ldh - 1) return;
    }
    __shared__ A wl[kChunk];
    __shared__ double red[kBT / kWave];
    const TS* w = static_cast<const TS*>(from_x0 ? d.x0 : d.w);
    const int64_t n = d.n;
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
    if (threadIdx.x == 0) d.pnrm[blockIdx.x] = t;
    __syncthreads();
    chunk_dots(static_cast<const TS*>(d.V), d.ldv, p, wl, base, n, d.partial);
}

// Reduction of the nblk partial dots of the kDotU coefficients i0 + stride u
// by one wavefront: per coefficient, lanes over blocks in a fixed order, then a
// shuffle tree, so every block of a fused pass gets the same bits.  The loads
// of the kDotU coefficients overlap.  REAL: the partials are stored as doubles
// (real states), the imaginary parts of the results exact zeros.
template <bool REAL>
__device__ inline void reduce_coefs(const double2* __restrict__ partial, int nblk, int p, int i0, int stride,
                                   int lane, double2 (&out)[kDotU]) {
    double2 sv[kDotU];
#pragma unroll
    for (int u = 0; u < kDotU; ++u) sv[u] = cmk<double2>(0.0, 0.0);
    for (int b = lane; b < nblk; b += kWave) {
        double2 t[kDotU];
#pragma unroll
        for (int u = 0; u < kDotU; ++u) {
            const int i = i0 + stride * u;  // i >= p: a valid entry, result unused
            const int64_t at = int64_t(b) * p + (i < p ? i : p - 1);
            if constexpr (REAL)
                t[u] = cmk<double2>(ldg(reinterpret_cast<const double*>(partial), at), 0.0);
            else
                t[u] = ldg(partial, at);
        }
#pragma unroll
        for (int u = 0; u < kDotU; ++u) sv[u] = cadd(sv[u], t[u]);
    }
#pragma unroll
    for (int u = 0; u < kDotU; ++u) out[u] = wave_sum(sv[u]);
}
__device__ inline double reduce_norm(const double* __restrict__ pn, int nblk, int lane) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += kWave) s += pn[b];
    return wave_sum(s);
}

// beta_j = ||w64|| from the pass-2 chunk norms, v_{j+1} = w64 / beta_j; block
// blk == 0 of an instance records H[j+1][j], beta and the breakdown /
// non-finite flags; blocks blk of nb scale a grid-stride share of the vector.
template <typename TS> __device__ inline void finalize_scale(const KryDesc& d, int j, int blk, int nb) {
    using A = typename ET<TS>::A;
    __shared__ double sb;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (wave == 0) {
        const double s = reduce_norm(d.pnrm, d.nblk, lane);
        if (lane == 0) {
            const double beta = sqrt(s);
            sb = beta;
            if (blk == 0) {
                const double win = sqrt(d.scal[1]);
                d.H[size_t(d.ldh) * j + (j + 1)] = cmk<double2>(beta, 0.0);
                d.scal[2] = beta;
                d.rr->beta = beta;
                d.rr->w_in = win;
                d.rr->nonfinite = !(isfinite(beta) && isfinite(win));
                d.rr->breakdown = (beta <= 64.0 * 2.220446049250313e-16 * win) ? 1 : 0;
                if (d.rr->breakdown && d.rr->bd_step == 0) d.rr->bd_step = j + 1;
            }
        }
    }
    __syncthreads();
    const double b = sb;
    const double inv = (b > 0.0 && isfinite(b)) ? 1.0 / b : 0.0;
    TS* v = static_cast<TS*>(d.V) + (j + 1) * d.ldv;
    const A* w64 = static_cast<const A*>(d.w64);
    // eight loads in flight before their stores (one block scales a whole short
    // state when the normalisation is fused into pass 2)
    constexpr int U = 8;
    const int64_t st = int64_t(nb) * blockDim.x;
    int64_t g = int64_t(blk) * blockDim.x + threadIdx.x;
    for (; g + (U - 1) * st < d.n; g += U * st) {
        A x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = w64[g + u * st];
#pragma unroll
        for (int u = 0; u < U; ++u) v[g + u * st] = ET<TS>::store(scale_by(x[u], inv));
    }
    for (; g < d.n; g += st) v[g] = ET<TS>::store(scale_by(w64[g], inv));
}

// The coefficients of a Gram-Schmidt pass from the partial dots of the kernel
// before it (pass 1: partial, pass 2: partial2): waves w0, w0 + wstride, ...
// of the caller each take kDotU coefficients i = i0 + 4u; hl (if not null)
// receives them; write_h: H column j (pass 1: = h, pass 2: += h) and d.h;
// pass 1 with write_h also stores ||w||^2 from the chunk norms in scal[1].
template <typename TS>
__device__ inline void reduce_pass_coefs(const KryDesc& d, int p, int j, int pass, double2* hl, bool write_h,
                                         bool norm, int w0, int lane, int wave_of, int wstride) {
    const double2* pin = pass == 1 ? d.partial : d.partial2;
    double2* Hcol = d.H + size_t(d.ldh) * j;
    constexpr int NW = kBT / kWave;
    for (int i0 = w0; i0 < p; i0 += wstride * kDotU) {
        double2 sv[kDotU];
        reduce_coefs<!std::is_same<TS, double2>::value>(pin, d.nblk, p, i0, NW, lane, sv);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < kDotU; ++u) {
                const int i = i0 + NW * u;
                if (i < p) {
                    if (hl) hl[i] = sv[u];
                    if (write_h) {
                        Hcol[i] = pass == 1 ? sv[u] : cadd(Hcol[i], sv[u]);
                        d.h[i] = sv[u];
                    }
                }
            }
        }
    }
    if (pass == 1 && norm && wave_of == 0) {
        const double s = reduce_norm(d.pnrm, d.nblk, lane);
        if (lane == 0) d.scal[1] = s;
    }
}

// Long states: the coefficients of a pass reduced once, by ceil(p / 16)
// workgroups per instance (each wave kDotU of them, in the order the fused
// passes use), instead of by every block of the pass.
template <typename TS>
__global__ __launch_bounds__(kBT) void k_reduce_coefs(const KryDesc* __restrict__ Dv, int p, int j, int pass) {
    const KryDesc& d = Dv[blockIdx.y];
    if (!d.active) return;
    p += d.poff;
    j += d.poff;
    if (j >= d.ldh - 1) return;
    constexpr int NW = kBT / kWave;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // block b, wave w: coefficients b * NW * kDotU + w + NW u
    const int base = int(blockIdx.x) * NW * kDotU;
    reduce_pass_coefs<TS>(d, p, j, pass, nullptr, true, blockIdx.x == 0, base + wave, lane, wave,
                          int(gridDim.x) * NW);
}

// One Gram-Schmidt pass of step j with the reduction of the previous kernel's
// partial dots folded in (every block reduces them itself; block 0 writes H):
//   pass 1: h1 from partial (k_dot), H[.][j] = h1, scal[1] = ||w||^2 from pnrm;
//           w64 = w - V h1; chunk norms -> pnrm2, dots V^H w64 -> partial2.
//   pass 2: h2 from partial2, H[.][j] += h2; w64 -= V h2; chunk norms -> pnrm.
// The buffers alternate so that no block overwrites partial sums another block
// still reads.
template <typename TS>
__global__ __launch_bounds__(kBT) void k_cgs_pass(const KryDesc* __restrict__ Dv, int p, int j, int pass,
                                                  int fuse_final, int pre_reduced) {
    using A = typename ET<TS>::A;
    const KryDesc& d = Dv[blockIdx.y];
    if (!d.active || int(blockIdx.x) >= d.nblk) return;
    p += d.poff;
    j += d.poff;
    if (j >= d.ldh - 1) return;
    __shared__ A wl[kChunk];
    __shared__ double2 hl[kMaxKrylov + 1];
    __shared__ double red[kBT / kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (pre_reduced) {
        // k_reduce_coefs has reduced the coefficients into h (and written H)
        for (int i = threadIdx.x; i < p; i += kBT) hl[i] = d.h[i];
    } else {
        reduce_pass_coefs<TS>(d, p, j, pass, hl, int(blockIdx.x) == 0, int(blockIdx.x) == 0, wave, lane,
                              wave, kBT / kWave);
    }
    __syncthreads();
    const TS* V = static_cast<const TS*>(d.V);
    const TS* w_in = static_cast<const TS*>(d.w);
    A* w64 = static_cast<A*>(d.w64);  // read and written in place
    const int64_t n = d.n, ldv = d.ldv;
    const int64_t base = int64_t(blockIdx.x) * kChunk;
    const int64_t g0 = base + threadIdx.x;
    A x[kEPT];
    bool ok[kEPT];
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
        const int64_t g = g0 + e * kBT;
        ok[e] = g < n;
        x[e] = zero_of<A>();
        if (ok[e]) x[e] = pass == 1 ? ET<TS>::acc(w_in[g]) : w64[g];
    }
    project_out<kEPT>(x, V, ldv, g0, n, hl, p);
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
        if (!ok[e]) x[e] = zero_of<A>();
        if (ok[e]) w64[g0 + e * kBT] = x[e];
        wl[threadIdx.x + e * kBT] = x[e];
        s2 += nrm2(x[e]);
    }
    double t = block_sum(s2, red);
    if (threadIdx.x == 0) (pass == 1 ? d.pnrm2 : d.pnrm)[blockIdx.x] = t;
    if (pass == 1) {
        __syncthreads();
        chunk_dots(V, ldv, p, wl, base, n, d.partial2);
    } else if (fuse_final) {
        // the last block of the instance to finish does the normalisation: every
        // thread publishes its stores device-wide, one thread counts the block in
        __shared__ int last;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(cgs_counter(d), 1) == d.nblk - 1;
        __syncthreads();
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other blocks' w64 and norms
            if (threadIdx.x == 0) *cgs_counter(d) = 0;            // for the next step
            finalize_scale<TS>(d, j, 0, 1);
        }
    }
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_scale_final(const KryDesc* __restrict__ Dv, int j) {
    const KryDesc& d = Dv[blockIdx.y];
    if (!d.active) return;
    j += d.poff;
    if (j >= d.ldh - 1) return;
    finalize_scale<TS>(d, j, int(blockIdx.x), int(gridDim.x));
}

// One wavefront per instance: scal[slot] = sum of the nblk chunk norms (lanes
// over blocks in a fixed order, then a shuffle tree).
__global__ __launch_bounds__(kWave) void k_reduce_norm(const KryDesc* __restrict__ Dv, int slot) {
    const KryDesc& d = Dv[blockIdx.x];
    if (!d.active) return;
    const double s = reduce_norm(d.pnrm, d.nblk, threadIdx.x);
    if (threadIdx.x == 0) d.scal[slot] = s;
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_scale(const KryDesc* __restrict__ Dv, int j) {
    using A = typename ET<TS>::A;
    const KryDesc& d = Dv[blockIdx.y];
    if (!d.active) return;
    TS* V = static_cast<TS*>(d.V);
    const int64_t n = d.n;
    if (j >= 0) {
        const double b = d.scal[2];
        const double inv = (b > 0.0 && isfinite(b)) ? 1.0 / b : 0.0;
        const A* w64 = static_cast<const A*>(d.w64);
        TS* v = V + (j + 1) * d.ldv;
        for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
            v[g] = ET<TS>::store(scale_by(w64[g], inv));
    } else {
        const double s2 = d.scal[0];
        const double inv = (s2 > 0.0 && isfinite(s2)) ? 1.0 / sqrt(s2) : 0.0;
        const TS* x = static_cast<const TS*>(d.x0);
        for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += int64_t(gridDim.x) * blockDim.x)
            V[g] = ET<TS>::store(scale_by(ET<TS>::acc(x[g]), inv));
    }
}

template <typename TS>
__global__ __launch_bounds__(kBT) void k_ritz(const KryDesc* __restrict__ Dv) {
    const KryDesc& d = Dv[blockIdx.z];
    const int s = blockIdx.y;
    if (!d.ritz || s >= d.rr->nsel) return;
    const int p = d.steps;
    const TS* V = static_cast<const TS*>(d.V);
    const double2* y = d.Y + size_t(s) * p;  // unit Ritz coordinates of wanted pair s
    double2* X = static_cast<double2*>(d.ritz);
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < d.n; g += int64_t(gridDim.x) * blockDim.x) {
        double2 acc = cmk<double2>(0.0, 0.0);
        for (int i = 0; i < p; ++i) acc = cadd(acc, cgain(y[i], ET<TS>::acc(V[i * d.ldv + g])));
        X[size_t(s) * d.n + g] = acc;
    }
}

__global__ void k_gather(const KryDesc* __restrict__ Dv, int k) {
    // out: [mu re,im]*k | [lambda re,im]*k | [res]*k, zero beyond nsel
    const KryDesc& d = Dv[blockIdx.x];
    const int s = threadIdx.x;
    if (s >= k) return;
    const int nsel = d.rr->nsel;
    double* out = d.out;
    if (s >= nsel) {
        out[2 * s] = out[2 * s + 1] = 0.0;
        out[2 * k + 2 * s] = out[2 * k + 2 * s + 1] = 0.0;
        out[4 * k + s] = 0.0;
        return;
    }
    const int i = d.sel[s];
    const double2 m = d.mu[i];
    out[2 * s] = m.x;
    out[2 * s + 1] = m.y;
    out[2 * k + 2 * s] = log(hypot(m.x, m.y)) / d.T;
    out[2 * k + 2 * s + 1] = atan2(m.y, m.x) / d.T;
    out[4 * k + s] = d.res[i];
}

// Krylov-Schur truncation (Sec. 3.2.2, step 4) of a real basis: Vout_c =
// sum_{j<m} V_j W[j + m c] for c < kp, and Vout_kp = V_m (v_{p+1} = v_{m+1}).  W
// (FP64, m x kp, column-major) is staged in LDS by tiles of kRotCols output
// vectors (blockIdx.y); each thread owns one element index, streams its m
// coalesced basis entries once per tile and accumulates in FP64.
constexpr int kRotCols = 16;
template <typename TS>
__global__ __launch_bounds__(kBT) void k_rotate(const TS* __restrict__ Vin, TS* __restrict__ Vout,
                                                const double* __restrict__ W, int64_t n, int64_t ldv, int m, int kp) {
    __shared__ double Ws[kMaxKrylov * kRotCols];
    const int c0 = blockIdx.y * kRotCols;
    for (int e = threadIdx.x; e < m * kRotCols; e += kBT) {
        const int j = e / kRotCols, c = e % kRotCols;
        Ws[e] = (c0 + c < kp) ? W[j + size_t(m) * (c0 + c)] : 0.0;
    }
    __syncthreads();
    for (int64_t g = int64_t(blockIdx.x) * kBT + threadIdx.x; g < n; g += int64_t(gridDim.x) * kBT) {
        double acc[kRotCols];
#pragma unroll
        for (int c = 0; c < kRotCols; ++c) acc[c] = 0.0;
        for (int j = 0; j < m; ++j) {
            const double x = ET<TS>::acc(Vin[j * ldv + g]);
#pragma unroll
            for (int c = 0; c < kRotCols; ++c) acc[c] = fma(x, Ws[j * kRotCols + c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < kRotCols; ++c)
            if (c0 + c < kp) Vout[(c0 + c) * ldv + g] = ET<TS>::store(acc[c]);
        if (blockIdx.y == 0) Vout[kp * ldv + g] = Vin[m * ldv + g];
    }
}

inline int grid_for(int64_t n, int cap) {
    int64_t b = (n + kBT - 1) / kBT;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return int(b);
}

}  // namespace

template <typename TS>
void launch_check_finite(const KryDesc* D, int count, int64_t nmax, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite<TS>, dim3(grid_for(nmax, 1024), count), dim3(kBT), 0, s, D);
}

template <typename TS>
void launch_dot(const KryDesc* D, int count, int nblk_max, int p, bool from_x0, hipStream_t s) {
    hipLaunchKernelGGL(k_dot<TS>, dim3(nblk_max, count), dim3(kBT), 0, s, D, p, from_x0 ? 1 : 0);
}

void launch_reduce_norm(const KryDesc* D, int count, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_norm, dim3(count), dim3(kWave), 0, s, D, slot);
}

template <typename TS>
void launch_cgs_pass(const KryDesc* D, int count, int nblk_max, int p, int j, int pass, bool fuse_final,
                     hipStream_t s, int pextra) {
    const bool pre = nblk_max >= kPreReduceMinBlocks;  // long states: one reduction launch first
    if (pre) {
        // pextra: the largest step offset of the batch (its instances reduce up to p + pextra coefficients)
        constexpr int per_block = (kBT / kWave) * kDotU;
        hipLaunchKernelGGL(k_reduce_coefs<TS>, dim3((p + pextra + per_block - 1) / per_block, count), dim3(kBT), 0,
                           s, D, p, j, pass);
    }
    hipLaunchKernelGGL(k_cgs_pass<TS>, dim3(nblk_max, count), dim3(kBT), 0, s, D, p, j, pass, fuse_final ? 1 : 0,
                       pre ? 1 : 0);
}

template <typename TS>
void launch_scale_final(const KryDesc* D, int count, int64_t nmax, int j, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_final<TS>, dim3(grid_for(nmax, 1024), count), dim3(kBT), 0, s, D, j);
}

template <typename TS>
void launch_scale(const KryDesc* D, int count, int64_t nmax, int j, hipStream_t s) {
    hipLaunchKernelGGL(k_scale<TS>, dim3(grid_for(nmax, 1024), count), dim3(kBT), 0, s, D, j);
}

template <typename TS>
void launch_ritz_vectors(const KryDesc* D, int count, int64_t nmax, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_ritz<TS>, dim3(grid_for(nmax, 1024), k, count), dim3(kBT), 0, s, D);
}

void launch_gather(const KryDesc* D, int count, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(count), dim3(128), 0, s, D, k);
}

template <typename TS>
void launch_rotate(const void* Vin, void* Vout, const double* W, int64_t n, int64_t ldv, int m, int kp, hipStream_t s) {
    hipLaunchKernelGGL(k_rotate<TS>, dim3(grid_for(n, 1024), (kp + kRotCols - 1) / kRotCols), dim3(kBT), 0, s,
                       static_cast<const TS*>(Vin), static_cast<TS*>(Vout), W, n, ldv, m, kp);
}
template void launch_rotate<double>(const void*, void*, const double*, int64_t, int64_t, int, int, hipStream_t);
template void launch_rotate<float>(const void*, void*, const double*, int64_t, int64_t, int, int, hipStream_t);

#define TSK_INST(TS)                                                                                 \
    template void launch_check_finite<TS>(const KryDesc*, int, int64_t, hipStream_t);               \
    template void launch_dot<TS>(const KryDesc*, int, int, int, bool, hipStream_t);                  \
    template void launch_scale<TS>(const KryDesc*, int, int64_t, int, hipStream_t);                  \
    template void launch_cgs_pass<TS>(const KryDesc*, int, int, int, int, int, bool, hipStream_t, int); \
    template void launch_scale_final<TS>(const KryDesc*, int, int64_t, int, hipStream_t);             \
    template void launch_ritz_vectors<TS>(const KryDesc*, int, int64_t, int, hipStream_t);
TSK_INST(double)
TSK_INST(float)
TSK_INST(double2)
#undef TSK_INST

}  // namespace tsk
