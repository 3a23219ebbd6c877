// Shared device/host helpers of libtsk: complex arithmetic on HIP vector types,
// wavefront reductions and error plumbing.  gfx950 only (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/tsk.h"

namespace tsk {

constexpr int kWave = 64;

// ---- error plumbing (host) -------------------------------------------------
void set_error(const std::string& msg);
tsk_status fail(tsk_status st, const std::string& msg);

#define TSK_HIP(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::tsk::fail(TSK_EHIP, std::string(#expr) + ": " +               \
                                             hipGetErrorString(e_));               \
    } while (0)

#define TSK_TRY(expr)                                                              \
    do {                                                                           \
        tsk_status s_ = (expr);                                                    \
        if (s_ < 0) return s_;                                                     \
    } while (0)

// ---- complex helpers (device + host) ----------------------------------------
template <typename real> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename real> using cplx = typename cplx_t<real>::type;

template <typename C> __host__ __device__ inline C cmk(decltype(C{}.x) a, decltype(C{}.x) b) {
    C r; r.x = a; r.y = b; return r;
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename C> __host__ __device__ inline C cmulc(C a, C b) {
    return cmk<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __host__ __device__ inline C cscale(C a, decltype(C{}.x) s) { return cmk<C>(a.x * s, a.y * s); }
template <typename C> __host__ __device__ inline C cconj(C a) { return cmk<C>(a.x, -a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double cabs(double2 a) { return hypot(a.x, a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm (robust complex division)
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return cmk<double2>((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.y + b.x * r;
        return cmk<double2>((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ inline double2 csqrt(double2 z) {
    double r = hypot(z.x, z.y);
    if (r == 0.0) return cmk<double2>(0.0, 0.0);
    double t = sqrt(0.5 * (r + fabs(z.x)));
    if (z.x >= 0.0) return cmk<double2>(t, z.y / (2.0 * t));
    return cmk<double2>(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

// ---- splitmix64 (Steele, Lea & Flood, OOPSLA 2014), counter form ----------------
// Output i of the stream seeded with `seed`.
__host__ __device__ inline uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
// ---- LDS ordering inside one wavefront ------------------------------------------
// The LDS instructions of one wavefront execute in issue order, so lanes of a
// workgroup that is a single wavefront exchange data through LDS without a
// hardware barrier.  A wavefront-scope fence keeps the compiler from moving LDS
// accesses across the exchange point and needs no wait for outstanding stores.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// ---- wavefront reductions (device) -------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}
__device__ inline double2 wave_sum(double2 v) {
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    return v;
}

// Device info shared with the host loop of the Arnoldi driver.
struct RitzResult {
    int done;          // first k accepted all converged
    int nsel;          // number of accepted Ritz values written (<= k)
    int nconv;         // accepted and converged
    int eig_fail;      // Hessenberg QR did not converge
    int breakdown;     // beta <= 64 eps ||w_in||
    int nonfinite;     // beta or H not finite
    int iters;         // QR iterations used
    int bd_step;       // first step order j+1 whose beta broke down (0: none); sticky
    int kept;          // Krylov-Schur contraction: order p kept (0: no contraction)
    int pad;
    double beta;
    double w_in;
};

constexpr int kMaxKrylov = 96;

}  // namespace tsk
