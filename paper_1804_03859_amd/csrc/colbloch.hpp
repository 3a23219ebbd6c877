// Column time stepper at N = 128 for a base profile of period 2 pi / 4 in y
// (the Kolmogorov flow U = sin 4y): the y-translation by a quarter period
// commutes with the linearized operator, so each kx column splits into four
// independent Bloch sectors, sector r holding the modes ky = 4 m + r.
//
// The pseudo-spectral product of the column with the profile restricted to one
// sector is exact on a 32-point grid.  Write the 128-point grid index as
// l = 32 a + b: the profile depends on b only, and the sector's field is
// g(y_l) = e^{i r y_l} G_r(b), G_r the 32-point inverse DFT of the sector's
// coefficients ĝ_{4m+r}.  The phase e^{i r y_l} cancels between the inverse
// and the forward transform, so the 128-point product restricted to the sector
// is p̂_{4m+r} = (1/32) sum_b U(y_b) G_r(b) e^{-2 pi i m b / 32}.  With the
// 2/3-dealiased modes (|ky| <= 42, at most 22 per sector) and a profile of one
// harmonic in b, the product spans fewer than 32 values of m, so no term wraps
// onto a kept mode: the result equals the 128-point pseudo-spectral product to
// rounding.  The base profile's period and harmonic content are checked on the
// host before this stepper is chosen.
//
// One 64-lane workgroup holds two sectors of one column (lanes 0..31 and
// 32..63), one mode per lane in natural DFT order, for the whole matvec.  The
// 32-point transforms are five radix-2 levels across the lanes of a half
// (partner lane ^ h): h = 16 a permlane16 swap, h = 8, 4 DPP row shifts under
// complementary bank masks, h = 2, 1 DPP quad permutations.  The inverse is
// decimation in frequency (natural order in, lane nu holding grid point
// bitrev5(nu) out) and the forward its transpose (decimation in time), so the
// grid side is read in the permuted order and nothing is reordered.
#pragma once

#include "colstep.hpp"

namespace tsk {

__device__ inline int bitrev5(int x) { return int(__builtin_bitreverse32(unsigned(x)) >> 27); }

// Value of lane (lane ^ H), H <= 16, of a 32-bit register (whole wavefront active).
template <int H> __device__ inline unsigned half_xor_u32(unsigned x, int lane) {
    if constexpr (H == 1 || H == 2) {
        return lane_xor_u32<H>(x);
    } else if constexpr (H == 4 || H == 8) {
        // lanes with bit H set read lane - H (row_shr), the others lane + H (row_shl)
        const unsigned a = unsigned(__builtin_amdgcn_mov_dpp(int(x), H == 8 ? 0x118 : 0x114, 0xF, H == 8 ? 0xC : 0xA,
                                                             false));
        return unsigned(__builtin_amdgcn_update_dpp(int(a), int(x), H == 8 ? 0x108 : 0x104, 0xF, H == 8 ? 0x3 : 0x5,
                                                    false));
    } else {
        static_assert(H == 16, "partner within a 32-lane half");
        // odd 16-lane rows of the first operand swap with the even rows of the
        // second: with both = x the partner sits in [0] on odd rows, in [1] on even rows
        const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? p[0] : p[1];
    }
}
template <int H> __device__ inline double half_xor(double v, int lane) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = half_xor_u32<H>(unsigned(b & 0xffffffffull), lane);
    const unsigned hi = half_xor_u32<H>(unsigned(b >> 32), lane);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int H> __device__ inline float half_xor(float v, int lane) {
    return __uint_as_float(half_xor_u32<H>(__float_as_uint(v), lane));
}
template <int H, typename C> __device__ inline C half_xor_c(C v, int lane) {
    return cmk<C>(half_xor<H>(v.x, lane), half_xor<H>(v.y, lane));
}

// Masked level twiddles of the 32-point DFT (forward sign), level h = 1 << l:
// e^{-2 pi i (nu mod h) / (2h)} on lanes with bit h of nu set, 1 on the others.
template <typename C> struct BlochTw {
    C lv[5];
    __device__ void load(const C* tw128, int nu) {  // tw128[t] = e^{-2 pi i t / 128}
#pragma unroll
        for (int l = 0; l < 5; ++l) {
            const int h = 1 << l;
            lv[l] = (nu & h) ? tw128[(nu & (h - 1)) * (128 / (2 * h))] : cmk<C>(1, 0);
        }
    }
};

template <int H, int SIGN, typename C> __device__ inline C bloch_dif(C v, const C& w, int lane) {
    using R = decltype(C{}.x);
    const R sg = (lane & H) ? R(-1) : R(1);
    const C p = half_xor_c<H>(v, lane);
    const C t = cmk<C>(p.x + sg * v.x, p.y + sg * v.y);
    return H == 1 ? t : cmul(t, tw_sign<SIGN>(w));
}
template <int H, int SIGN, typename C> __device__ inline C bloch_dit(C v, const C& w, int lane) {
    using R = decltype(C{}.x);
    const R sg = (lane & H) ? R(-1) : R(1);
    const C z = H == 1 ? v : cmul(v, tw_sign<SIGN>(w));
    const C p = half_xor_c<H>(z, lane);
    return cmk<C>(p.x + sg * z.x, p.y + sg * z.y);
}
// inverse (natural -> bitrev5 order) and forward (bitrev5 -> natural) 32-point DFTs
template <typename C> __device__ inline C bloch_inv(C v, const BlochTw<C>& t, int lane) {
    v = bloch_dif<16, +1>(v, t.lv[4], lane);
    v = bloch_dif<8, +1>(v, t.lv[3], lane);
    v = bloch_dif<4, +1>(v, t.lv[2], lane);
    v = bloch_dif<2, +1>(v, t.lv[1], lane);
    return bloch_dif<1, +1>(v, t.lv[0], lane);
}
template <typename C> __device__ inline C bloch_fwd(C v, const BlochTw<C>& t, int lane) {
    v = bloch_dit<1, -1>(v, t.lv[0], lane);
    v = bloch_dit<2, -1>(v, t.lv[1], lane);
    v = bloch_dit<4, -1>(v, t.lv[2], lane);
    v = bloch_dit<8, -1>(v, t.lv[3], lane);
    return bloch_dit<16, -1>(v, t.lv[4], lane);
}

// Grid: block 0 the kx = 0 column (diffusion only), block 1 + 2 (kx - 1) + h the
// sectors 2h, 2h + 1 of column kx (1 <= kx <= M).  Lawson RK4 as k_colstep.
template <typename real>
__global__ __launch_bounds__(kWave) void k_colstep_bloch(ColInst<real> I, const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    using G = Geo<128>;
    constexpr int M = G::M, P = 4, L = 32;
    const int lane = threadIdx.x;
    const real* __restrict__ xin = I.xbase;
    real* __restrict__ yout = I.y;
    const double alpha = I.alpha, Re = I.Re, dt = I.dt, cprop = I.cprop;
    const int nsteps = I.nsteps;
    if (blockIdx.x == 0) {
        // kx = 0: the advection term vanishes (d/dx of a y-only field)
        for (int q = lane; q < M; q += kWave) {
            const double jy = q + 1;
            const real E1 = real(exp(-jy * jy * dt / Re));
            real re = xin[2 * q], im = xin[2 * q + 1];
            for (int st = 0; st < nsteps; ++st) { re *= E1; im *= E1; }
            yout[2 * q] = re;
            yout[2 * q + 1] = im;
        }
        return;
    }
    const int kx = 1 + (int(blockIdx.x) - 1) / 2;
    const int r = 2 * ((int(blockIdx.x) - 1) % 2) + (lane >> 5);  // sector
    const int nu = lane & (L - 1);                                 // DFT index in the sector
    const int m = nu < L / 2 ? nu : nu - L;
    const int jy = P * m + r;
    const bool kp = jy >= -M && jy <= M;
    const int q = kp ? jy + M : 0;
    const double kxv = alpha * kx;
    const double K2 = kxv * kxv + double(jy) * jy;
    const real E1 = kp ? real(exp(-K2 * dt / Re)) : real(0);
    const real Eh = kp ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
    const real g1 = kp ? real(kxv * (1.0 - cprop / K2)) : real(0);
    const real kmask = kp ? real(1.0 / L) : real(0);
    const real nuv = I.negU[bitrev5(nu)];  // profile at the grid point this lane holds after the inverse
    const real* xs = xin + G::seg(kx);
    C w = kp ? cmk<C>(xs[2 * q], xs[2 * q + 1]) : cmk<C>(real(0), real(0));
    C acc = w, s = w;
    BlochTw<C> tw;
    tw.load(twg, nu);
    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);

    for (int st = 0; st < nsteps; ++st) {
        s = w;
#pragma unroll 4
        for (int stage = 0; stage < 4; ++stage) {
            C v = cmk<C>(-g1 * s.y, g1 * s.x);  // i kx (1 - c / K^2) s
            v = bloch_inv(v, tw, lane);
            C pr = cmk<C>(nuv * v.x, nuv * v.y);
            pr = bloch_fwd(pr, tw, lane);
            const C nh = cmk<C>(pr.x * kmask, pr.y * kmask);
            if (stage == 0) {
                acc = cmk<C>(E1 * (w.x + h6 * nh.x), E1 * (w.y + h6 * nh.y));
                s = cmk<C>(Eh * (w.x + h2 * nh.x), Eh * (w.y + h2 * nh.y));
            } else if (stage == 1) {
                acc.x += h3 * Eh * nh.x;
                acc.y += h3 * Eh * nh.y;
                s = cmk<C>(Eh * w.x + h2 * nh.x, Eh * w.y + h2 * nh.y);
            } else if (stage == 2) {
                acc.x += h3 * Eh * nh.x;
                acc.y += h3 * Eh * nh.y;
                s = cmk<C>(E1 * w.x + hh * Eh * nh.x, E1 * w.y + hh * Eh * nh.y);
            } else {
                w = cmk<C>(acc.x + h6 * nh.x, acc.y + h6 * nh.y);
            }
        }
    }
    real* ys = yout + G::seg(kx);
    if (kp) {
        ys[2 * q] = w.x;
        ys[2 * q + 1] = w.y;
    }
}

}  // namespace tsk
