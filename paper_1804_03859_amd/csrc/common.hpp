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
// ---- cross-lane exchange and wavefront reductions (device) ---------------------
__device__ inline int lane_id() { return int(__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u))); }

// Value of lane (lane ^ H), H <= 32, of a 32-bit register; the whole wavefront
// must be active.  H = 1, 2: DPP quad permutations; H = 4, 8: lanes with bit H
// set read lane - H (row_shr), the others lane + H (row_shl), under
// complementary bank masks; H = 16, 32: the gfx950 permlane swaps with both
// operands x (the first operand's odd 16-lane rows / upper half trade places
// with the second's even rows / lower half, so the partner sits in [0] on lanes
// with bit H set and in [1] on the others).
template <int H> __device__ inline unsigned xor_lane_u32(unsigned x, int lane) {
    if constexpr (H == 1 || H == 2) {
        return unsigned(__builtin_amdgcn_mov_dpp(int(x), H == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false));
    } else if constexpr (H == 4 || H == 8) {
        const unsigned a = unsigned(__builtin_amdgcn_mov_dpp(int(x), H == 8 ? 0x118 : 0x114, 0xF, H == 8 ? 0xC : 0xA,
                                                             false));
        return unsigned(__builtin_amdgcn_update_dpp(int(a), int(x), H == 8 ? 0x108 : 0x104, 0xF, H == 8 ? 0x3 : 0x5,
                                                    false));
    } else if constexpr (H == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? p[0] : p[1];
    } else {
        static_assert(H == 32, "partner distance");
        const auto p = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return (lane & 32) ? p[0] : p[1];
    }
}
template <int H> __device__ inline double xor_lane(double v, int lane) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = xor_lane_u32<H>(unsigned(b & 0xffffffffull), lane);
    const unsigned hi = xor_lane_u32<H>(unsigned(b >> 32), lane);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int H> __device__ inline float xor_lane(float v, int lane) {
    return __uint_as_float(xor_lane_u32<H>(__float_as_uint(v), lane));
}

// For H = 16, 32: a permlane swap of a 32-bit word with itself returns, on both
// lanes of each pair (lane, lane ^ H), the lower lane's word in [0] and the upper
// lane's in [1].
template <int H> __device__ inline void swap_pair_u32(unsigned x, unsigned& lower, unsigned& upper) {
    static_assert(H == 16 || H == 32, "permlane distance");
    const auto p = H == 32 ? __builtin_amdgcn_permlane32_swap(x, x, false, false)
                           : __builtin_amdgcn_permlane16_swap(x, x, false, false);
    lower = p[0];
    upper = p[1];
}
template <int H> __device__ inline void swap_pair(double v, double& lower, double& upper) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    unsigned l0, u0, l1, u1;
    swap_pair_u32<H>(unsigned(u & 0xffffffffull), l0, u0);
    swap_pair_u32<H>(unsigned(u >> 32), l1, u1);
    lower = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(l1) << 32) | l0));
    upper = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(u1) << 32) | u0));
}
template <int H> __device__ inline void swap_pair(float v, float& lower, float& upper) {
    unsigned l, u;
    swap_pair_u32<H>(__float_as_uint(v), l, u);
    lower = __uint_as_float(l);
    upper = __uint_as_float(u);
}

// Butterfly sum over the wavefront (partners lane ^ 32, ^ 16, ..., ^ 1); every
// lane ends with the same total.  The whole wavefront must be active.
__device__ inline double wave_sum(double v) {
    const int lane = lane_id();
    double lo, up;
    swap_pair<32>(v, lo, up);
    v = lo + up;  // = v + partner on both lanes (addition commutes exactly)
    swap_pair<16>(v, lo, up);
    v = lo + up;
    v += xor_lane<8>(v, lane);
    v += xor_lane<4>(v, lane);
    v += xor_lane<2>(v, lane);
    v += xor_lane<1>(v, lane);
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
