// Cross-lane complex FFT of length 128 for one wavefront (two points per
// lane), used by the column steppers at N = 128 instead of LDS passes.
//
// Lane L holds the positions L and L + 64 on the natural side (registers a, b).
// With k = 2 m + q (q < 2, m < 64),
//     X[2 m + q] = sum_L e^{s 2 pi i L m / 64} [ e^{s 2 pi i L q / 128} (x[L] + (-1)^q x[L + 64]) ],
// an in-lane radix-2 butterfly and twiddle followed, for q = 0 and 1, by a
// 64-point DFT across the lanes: six radix-2 levels whose partners are lanes
// L and L ^ h (h = 32, 16, ..., 1).  No level touches LDS.
//
// Levels h = 32, 16, 8, 4 first exchange one lane bit with the register index
// (a "pair swap": lanes with bit h clear end up holding their own a and the
// partner's a, lanes with bit h set the partner's b and their own b), so each
// lane then has both inputs of one butterfly and computes both outputs
//     a' = a + b,  b' = (a - b) W,  W = e^{s 2 pi i (L mod h) / (2h)}.
// The swaps are one permlane32 / permlane16 swap per 32-bit word (gfx950) and,
// for h = 8 and 4, two DPP row shifts under complementary bank masks.  Levels
// h = 2, 1 exchange with the partner by DPP quad permutations and keep the
// register meaning:
//     p = x[L ^ h];  x = (p + sg x) W'   (sg = -1 if bit h set, else +1;
//                                         W' = W on lanes with bit h set, else 1)
//
// The inverse transform (decimation in frequency) takes natural order and
// leaves lane L, register r holding grid position 2 m + q with
//     q = bit 5 of L, m = (bit 4, bit 3, bit 2 of L, r, bit 1, bit 0 of L) from the
//     least significant bit up (xl_grid_pos).
// The forward transform is its exact transpose (decimation in time: the levels
// in reverse order, each butterfly transposed, the same self-inverse swaps,
// twiddles conjugated), so it takes that order and returns natural order.  A
// stepper that runs inverse -> pointwise product -> forward never reorders
// anything: it reads the grid-side profiles at the permuted positions.
#pragma once

#include "colfft.hpp"

namespace tsk {

template <int N> constexpr bool col_xl() { return N == 128 && ColPlan<N>::RE == 2 && ColPlan<N>::NB == kWave; }

// Grid position held by lane L, register r, after the inverse transform.
__device__ inline int xl_grid_pos(int lane, int r) {
    const int q = (lane >> 5) & 1;
    const int m = ((lane >> 4) & 1) | (((lane >> 3) & 1) << 1) | (((lane >> 2) & 1) << 2) | (r << 3) |
                  (((lane >> 1) & 1) << 4) | ((lane & 1) << 5);
    return 2 * m + q;
}

// ---- 32-bit exchanges (the whole wavefront active) ---------------------------------
// Partner value lane ^ H for H = 1, 2 (DPP quad permutations).
template <int H> __device__ inline unsigned lane_xor_u32(unsigned x) {
    static_assert(H == 1 || H == 2, "quad partners only");
    return unsigned(__builtin_amdgcn_mov_dpp(int(x), H == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false));
}

// Pair swap of lane bit H with the register index for one 32-bit word of a and b.
template <int H> __device__ inline void pair_swap_u32(unsigned& a, unsigned& b) {
    if constexpr (H == 32) {
        const auto p = __builtin_amdgcn_permlane32_swap(a, b, false, false);  // a.hi <-> b.lo
        a = p[0];
        b = p[1];
    } else if constexpr (H == 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(a, b, false, false);  // odd rows of a <-> even rows of b
        a = p[0];
        b = p[1];
    } else {
        static_assert(H == 8 || H == 4, "row-local distances");
        // set lanes (banks 2,3 for H = 8; banks 1,3 for H = 4) take b from lane - H;
        // clear lanes take the original a from lane + H
        const unsigned t = a;
        a = unsigned(__builtin_amdgcn_update_dpp(int(a), int(b), H == 8 ? 0x118 : 0x114, 0xF, H == 8 ? 0xC : 0xA,
                                                 false));
        b = unsigned(__builtin_amdgcn_update_dpp(int(b), int(t), H == 8 ? 0x108 : 0x104, 0xF, H == 8 ? 0x3 : 0x5,
                                                 false));
    }
}

template <int H> __device__ inline void pair_swap(double& a, double& b) {
    unsigned long long ua = static_cast<unsigned long long>(__double_as_longlong(a));
    unsigned long long ub = static_cast<unsigned long long>(__double_as_longlong(b));
    unsigned alo = unsigned(ua & 0xffffffffull), ahi = unsigned(ua >> 32);
    unsigned blo = unsigned(ub & 0xffffffffull), bhi = unsigned(ub >> 32);
    pair_swap_u32<H>(alo, blo);
    pair_swap_u32<H>(ahi, bhi);
    a = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(ahi) << 32) | alo));
    b = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(bhi) << 32) | blo));
}
template <int H> __device__ inline void pair_swap(float& a, float& b) {
    unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
    pair_swap_u32<H>(ua, ub);
    a = __uint_as_float(ua);
    b = __uint_as_float(ub);
}
template <int H, typename C> __device__ inline void pair_swap_c(C& a, C& b) {
    pair_swap<H>(a.x, b.x);
    pair_swap<H>(a.y, b.y);
}

template <int H> __device__ inline double lane_xor(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    const unsigned lo = lane_xor_u32<H>(unsigned(b & 0xffffffffull));
    const unsigned hi = lane_xor_u32<H>(unsigned(b >> 32));
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
template <int H> __device__ inline float lane_xor(float v) { return __uint_as_float(lane_xor_u32<H>(__float_as_uint(v))); }
template <int H, typename C> __device__ inline C lane_xor_c(C v) { return cmk<C>(lane_xor<H>(v.x), lane_xor<H>(v.y)); }

// Per-lane twiddles (forward sign; the inverse uses their conjugates).
template <typename C> struct XlTw {
    C in;     // e^{-2 pi i L / 128} (slot 1 of the in-lane step)
    C lv[6];  // level h = 1 << l: W for h >= 4, the masked W' for h = 2 (1 for h = 1)
    // tw[stride t] = e^{-2 pi i t / 128}, t < 128 (stride > 1: a finer table)
    __device__ void load(const C* tw, int lane, int stride = 1) {
        in = tw[stride * lane];
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            const int h = 1 << l;
            const C w = tw[stride * (lane & (h - 1)) * (128 / (2 * h))];
            lv[l] = (h >= 4 || (lane & h)) ? w : cmk<C>(1, 0);
        }
    }
};

template <int H, int SIGN, int COLS, typename C>
__device__ inline void xl_dif_swap(C (&v)[COLS][1][2], const C& w) {
    const C ws = tw_sign<SIGN>(w);
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        C a = v[c][0][0], b = v[c][0][1];
        pair_swap_c<H>(a, b);
        v[c][0][0] = cadd(a, b);
        v[c][0][1] = cmul(csub(a, b), ws);
    }
}
template <int H, int SIGN, int COLS, typename C>
__device__ inline void xl_dit_swap(C (&v)[COLS][1][2], const C& w) {
    const C ws = tw_sign<SIGN>(w);
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const C a = v[c][0][0], wb = cmul(v[c][0][1], ws);
        C na = cadd(a, wb), nb = csub(a, wb);
        pair_swap_c<H>(na, nb);
        v[c][0][0] = na;
        v[c][0][1] = nb;
    }
}
template <int H, int SIGN, int COLS, typename C>
__device__ inline void xl_dif_xor(C (&v)[COLS][1][2], const C& w, int lane) {
    using R = decltype(C{}.x);
    const R sg = (lane & H) ? R(-1) : R(1);
    const C ws = tw_sign<SIGN>(w);
#pragma unroll
    for (int c = 0; c < COLS; ++c)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const C p = lane_xor_c<H>(v[c][0][q]);
            const C t = cmk<C>(p.x + sg * v[c][0][q].x, p.y + sg * v[c][0][q].y);
            v[c][0][q] = H == 1 ? t : cmul(t, ws);  // W' = 1 on every lane for h = 1
        }
}
template <int H, int SIGN, int COLS, typename C>
__device__ inline void xl_dit_xor(C (&v)[COLS][1][2], const C& w, int lane) {
    using R = decltype(C{}.x);
    const R sg = (lane & H) ? R(-1) : R(1);
    const C ws = tw_sign<SIGN>(w);
#pragma unroll
    for (int c = 0; c < COLS; ++c)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const C z = H == 1 ? v[c][0][q] : cmul(v[c][0][q], ws);
            const C p = lane_xor_c<H>(z);
            v[c][0][q] = cmk<C>(p.x + sg * z.x, p.y + sg * z.y);
        }
}

// Inverse (SIGN = +1): natural order in, xl_grid_pos order out.
template <int COLS, typename C>
__device__ inline void xl_fft_inv(C (&v)[COLS][1][2], const XlTw<C>& t, int lane) {
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        dft<2, +1>(v[c][0]);
        v[c][0][1] = cmul(v[c][0][1], tw_sign<+1>(t.in));
    }
    xl_dif_swap<32, +1>(v, t.lv[5]);
    xl_dif_swap<16, +1>(v, t.lv[4]);
    xl_dif_swap<8, +1>(v, t.lv[3]);
    xl_dif_swap<4, +1>(v, t.lv[2]);
    xl_dif_xor<2, +1>(v, t.lv[1], lane);
    xl_dif_xor<1, +1>(v, t.lv[0], lane);
}

// Forward (SIGN = -1): xl_grid_pos order in, natural order out.
template <int COLS, typename C>
__device__ inline void xl_fft_fwd(C (&v)[COLS][1][2], const XlTw<C>& t, int lane) {
    xl_dit_xor<1, -1>(v, t.lv[0], lane);
    xl_dit_xor<2, -1>(v, t.lv[1], lane);
    xl_dit_swap<4, -1>(v, t.lv[2]);
    xl_dit_swap<8, -1>(v, t.lv[3]);
    xl_dit_swap<16, -1>(v, t.lv[4]);
    xl_dit_swap<32, -1>(v, t.lv[5]);
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        v[c][0][1] = cmul(v[c][0][1], tw_sign<-1>(t.in));
        dft<2, -1>(v[c][0]);
    }
}

}  // namespace tsk
