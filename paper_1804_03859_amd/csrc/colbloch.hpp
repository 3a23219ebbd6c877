// Column time stepper for N = 4L (L = 32, 64, 128) and a base profile of period
// 2 pi / 4 in y (the Kolmogorov flow U = sin 4y): the y-translation by a quarter
// period commutes with the linearized operator, so each kx column splits into
// four independent Bloch sectors, sector r holding the modes ky = 4 m + r.
//
// The pseudo-spectral product of the column with the profile restricted to one
// sector is exact on an L-point grid.  Write the N-point grid index as
// l = L a + b: the profile depends on b only, and the sector's field is
// g(y_l) = e^{i r y_l} G_r(b), G_r the L-point inverse DFT of the sector's
// coefficients ĝ_{4m+r}.  The phase e^{i r y_l} cancels between the inverse
// and the forward transform, so the N-point product restricted to the sector
// is p̂_{4m+r} = (1/L) sum_b U(y_b) G_r(b) e^{-2 pi i m b / L}.  With the
// 2/3-dealiased modes (|ky| < N/3, about 2L/3 per sector) and a profile of one
// harmonic in b, the product spans fewer than L values of m, so no term wraps
// onto a kept mode: the result equals the N-point pseudo-spectral product to
// rounding.  The base profile's period and harmonic content are checked on the
// host before this stepper is chosen.
//
// Lane layout, in natural DFT order, for the whole matvec (one sector per
// workgroup of one wavefront):
//   L = 32:  the real and imaginary parts of a mode on a lane pair
//            (k_colstep_bloch_split below); five radix-2 levels.
//   L = 64:  one mode per lane; six levels.
//   L = 128: two modes per lane; the 128-point cross-lane transform of
//            colxl.hpp.
// The levels exchange with the partner lane ^ h: h = 32, 16 by permlane swaps,
// h = 8, 4 by DPP row shifts under complementary bank masks, h = 2, 1 by DPP
// quad permutations (common.hpp).  The inverse is decimation in frequency (natural order
// in, bit-reversed grid positions out) and the forward its transpose
// (decimation in time), so the grid side is read in the permuted order and
// nothing is reordered.
#pragma once

#include "colstep.hpp"
#include "colxl.hpp"

namespace tsk {

__device__ inline int bitrev5(int x) { return int(__builtin_bitreverse32(unsigned(x)) >> 27); }

__device__ inline int bitrev6b(int x) { return int(__builtin_bitreverse32(unsigned(x)) >> 26); }

template <int H, typename C> __device__ inline C half_xor_c(C v, int lane) {
    return cmk<C>(xor_lane<H>(v.x, lane), xor_lane<H>(v.y, lane));
}

// Masked level twiddles of the 64-point DFT (forward sign), level h = 1 << l:
// e^{-2 pi i (nu mod h) / (2h)} on lanes with bit h of nu set, 1 on the others;
// twN[t] = e^{-2 pi i t / 256}.
template <typename C> struct BlochTw {
    C lv[6];
    __device__ void load(const C* twN, int nu) {
#pragma unroll
        for (int l = 0; l < 6; ++l) {
            const int h = 1 << l;
            lv[l] = (nu & h) ? twN[(nu & (h - 1)) * (256 / (2 * h))] : cmk<C>(1, 0);
        }
    }
};

// v + partner on the lower lane of the pair (lane, lane ^ H), partner - v on
// the upper one; for H = 16, 32 straight from the two results of a permlane swap.
template <int H, typename C> __device__ inline C bloch_bfly(C v, int lane) {
    using R = decltype(C{}.x);
    const R sg = (lane & H) ? R(-1) : R(1);
    if constexpr (H == 16 || H == 32) {
        R lx, ux, ly, uy;
        swap_pair<H>(v.x, lx, ux);
        swap_pair<H>(v.y, ly, uy);
        return cmk<C>(sg * ux + lx, sg * uy + ly);
    } else {
        const C p = half_xor_c<H>(v, lane);
        return cmk<C>(p.x + sg * v.x, p.y + sg * v.y);
    }
}
template <int H, int SIGN, typename C> __device__ inline C bloch_dif(C v, const C& w, int lane) {
    const C t = bloch_bfly<H>(v, lane);
    return H == 1 ? t : cmul(t, tw_sign<SIGN>(w));
}
template <int H, int SIGN, typename C> __device__ inline C bloch_dit(C v, const C& w, int lane) {
    const C z = H == 1 ? v : cmul(v, tw_sign<SIGN>(w));
    return bloch_bfly<H>(z, lane);
}
// inverse (natural -> bit-reversed order) and forward (bit-reversed -> natural)
// 64-point DFTs, one value per lane
template <typename C> __device__ inline C bloch_inv(C v, const BlochTw<C>& t, int lane) {
    v = bloch_dif<32, +1>(v, t.lv[5], lane);
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
    v = bloch_dit<16, -1>(v, t.lv[4], lane);
    return bloch_dit<32, -1>(v, t.lv[5], lane);
}

// Workgroups of a Bloch launch: the kx = 0 column, then the four sectors of
// every column kx >= 1, one per workgroup.
inline int bloch_blocks(int M) { return 1 + 4 * M; }

// L = 64 and 128.  Grid x (bloch_blocks): block 0 the kx = 0 column (diffusion
// only), then the sectors of column kx = 1..M.  Grid y: the instance, insts[ids[blockIdx.y]]
// of a batch (input of Arnoldi step jstep: xbase + jstep xstride; finished
// instances skip), or `one` when insts is null.  Lawson RK4 as k_colstep.
template <typename real, int L>
__global__ __launch_bounds__(kWave) void k_colstep_bloch(ColInst<real> one, const ColInst<real>* __restrict__ insts,
                                                         const int* __restrict__ ids, int jstep,
                                                         const cplx<real>* __restrict__ twg) {
    static_assert(L == 64 || L == 128, "sector length");
    using C = cplx<real>;
    constexpr int N = 4 * L;
    using G = Geo<N>;
    constexpr int M = G::M, P = 4;
    constexpr int S = L == 128 ? 2 : 1;  // modes per lane
    stepper_wave_priority();
    const ColInst<real>& I = insts ? insts[ids[blockIdx.y]] : one;
    if ((I.active && *I.active == 0) || jstep >= I.jmax) return;
    const int lane = threadIdx.x;
    const real* __restrict__ xin = I.xbase + jstep * I.xstride;
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
    const int b = int(blockIdx.x) - 1;
    const int kx = 1 + b / 4, r = b % 4;
    const double kxv = alpha * kx;
    const real* xs = xin + G::seg(kx);
    real E1[S], Eh[S], g1[S], kmask[S], nuv[S];
    int qs[S];
    bool kps[S];
    C w[S], acc[S], s[S];
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
        const int idx = lane + 64 * sl;  // DFT index in the sector
        const int m = idx < L / 2 ? idx : idx - L;
        const int jy = P * m + r;
        const bool kp = jy >= -M && jy <= M;
        kps[sl] = kp;
        qs[sl] = kp ? jy + M : 0;
        const double K2 = kxv * kxv + double(jy) * jy;
        E1[sl] = kp ? real(exp(-K2 * dt / Re)) : real(0);
        Eh[sl] = kp ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
        g1[sl] = kp ? real(kxv * (1.0 - cprop / K2)) : real(0);
        kmask[sl] = kp ? real(1.0 / L) : real(0);
        // profile at the grid point this slot holds after the inverse transform
        const int gpos = L == 64 ? bitrev6b(lane) : xl_grid_pos(lane, sl);
        nuv[sl] = I.negU[gpos];
        w[sl] = kp ? cmk<C>(xs[2 * qs[sl]], xs[2 * qs[sl] + 1]) : cmk<C>(real(0), real(0));
        acc[sl] = s[sl] = w[sl];
    }
    BlochTw<C> btw;
    XlTw<C> xtw;
    if constexpr (L == 128)
        xtw.load(twg, lane, N / 128);
    else
        btw.load(twg, lane);
    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);

    for (int st = 0; st < nsteps; ++st) {
#pragma unroll
        for (int sl = 0; sl < S; ++sl) s[sl] = w[sl];
#pragma unroll 4
        for (int stage = 0; stage < 4; ++stage) {
            C v[1][1][S];
#pragma unroll
            for (int sl = 0; sl < S; ++sl) v[0][0][sl] = cmk<C>(-g1[sl] * s[sl].y, g1[sl] * s[sl].x);  // i kx (1 - c/K^2) s
            if constexpr (L == 128)
                xl_fft_inv<1>(v, xtw, lane);
            else
                v[0][0][0] = bloch_inv(v[0][0][0], btw, lane);
#pragma unroll
            for (int sl = 0; sl < S; ++sl) v[0][0][sl] = cmk<C>(nuv[sl] * v[0][0][sl].x, nuv[sl] * v[0][0][sl].y);
            if constexpr (L == 128)
                xl_fft_fwd<1>(v, xtw, lane);
            else
                v[0][0][0] = bloch_fwd(v[0][0][0], btw, lane);
#pragma unroll
            for (int sl = 0; sl < S; ++sl) {
                const C nh = cmk<C>(v[0][0][sl].x * kmask[sl], v[0][0][sl].y * kmask[sl]);
                if (stage == 0) {
                    acc[sl] = cmk<C>(E1[sl] * (w[sl].x + h6 * nh.x), E1[sl] * (w[sl].y + h6 * nh.y));
                    s[sl] = cmk<C>(Eh[sl] * (w[sl].x + h2 * nh.x), Eh[sl] * (w[sl].y + h2 * nh.y));
                } else if (stage == 1) {
                    acc[sl].x += h3 * Eh[sl] * nh.x;
                    acc[sl].y += h3 * Eh[sl] * nh.y;
                    s[sl] = cmk<C>(Eh[sl] * w[sl].x + h2 * nh.x, Eh[sl] * w[sl].y + h2 * nh.y);
                } else if (stage == 2) {
                    acc[sl].x += h3 * Eh[sl] * nh.x;
                    acc[sl].y += h3 * Eh[sl] * nh.y;
                    s[sl] = cmk<C>(E1[sl] * w[sl].x + hh * Eh[sl] * nh.x, E1[sl] * w[sl].y + hh * Eh[sl] * nh.y);
                } else {
                    w[sl] = cmk<C>(acc[sl].x + h6 * nh.x, acc[sl].y + h6 * nh.y);
                }
            }
        }
    }
    real* ys = yout + G::seg(kx);
#pragma unroll
    for (int sl = 0; sl < S; ++sl)
        if (kps[sl]) {
            ys[2 * qs[sl]] = w[sl].x;
            ys[2 * qs[sl] + 1] = w[sl].y;
        }
}

// ---- 128^2: one sector per wavefront, real and imaginary parts on lane pairs ----------
// The 32-mode sectors of N = 128 with lane = 2 q + c: q the mode's DFT index
// (natural order), c = 0 the real part, c = 1 the imaginary part.  Every lane
// holds one real number, so an exchange moves two 32-bit words instead of four,
// the butterflies and the integrating-factor RK4 are one FP64 operation per
// lane, and a twiddle product needs the other part of the same mode (lane ^ 1):
//     (t W)_c = t_c Re W + t_(1-c) (c ? Im W : -Im W).
// The DFT levels h = 16 ... 1 pair lanes 2h apart; the inverse is decimation in
// frequency (lane q ends with grid position bitrev5(q)), the forward its
// transpose, as in the two-sectors-per-wavefront layout.
template <typename real> struct SplitTw {
    real wr[5], ws[5];  // level h = 1 << l: Re W', and (c ? Im W' : -Im W') for the forward W'
    real sg[5];         // butterfly sign: -1 on the lanes whose mode index has bit h set
    __device__ void load(const cplx<real>* twN, int q, int c) {
#pragma unroll
        for (int l = 0; l < 5; ++l) {
            const int h = 1 << l;
            const cplx<real> w = (q & h) ? twN[(q & (h - 1)) * (128 / (2 * h))] : cmk<cplx<real>>(1, 0);
            wr[l] = w.x;
            ws[l] = c ? w.y : -w.y;
            sg[l] = (q & h) ? real(-1) : real(1);
        }
    }
};

template <int H> constexpr int split_level() { return H == 16 ? 4 : H == 8 ? 3 : H == 4 ? 2 : H == 2 ? 1 : 0; }

// Butterfly sum/difference with the partner lane ^ B: the lower lane of the pair
// gets v + partner, the upper one partner - v (sg = -1 on upper lanes).  For
// B = 16, 32 a permlane swap of v with itself leaves (lower value, upper value)
// in its two results on both lanes of a pair, so no select is needed.
template <int B, typename real> __device__ inline real split_bfly(real v, real sg, int lane) {
    if constexpr (B == 16 || B == 32) {
        real lo, up;
        swap_pair<B>(v, lo, up);
        return sg * up + lo;
    } else {
        return sg * v + xor_lane<B>(v, lane);
    }
}
template <int H, typename real> __device__ inline real split_dif(real v, const SplitTw<real>& t, int lane) {
    constexpr int l = split_level<H>();
    const real tt = split_bfly<2 * H>(v, t.sg[l], lane);
    if constexpr (H == 1) return tt;
    return tt * t.wr[l] - xor_lane<1>(tt, lane) * t.ws[l];  // times conj(W')
}
template <int H, typename real> __device__ inline real split_dit(real v, const SplitTw<real>& t, int lane) {
    constexpr int l = split_level<H>();
    real z = v;
    if constexpr (H != 1) z = v * t.wr[l] + xor_lane<1>(v, lane) * t.ws[l];  // times W'
    return split_bfly<2 * H>(z, t.sg[l], lane);
}

// Grid as k_colstep_bloch (bloch_blocks(M) workgroups: kx = 0, then one sector
// per workgroup), N = 128 only.
template <typename real>
__global__ __launch_bounds__(kWave) void k_colstep_bloch_split(ColInst<real> one,
                                                               const ColInst<real>* __restrict__ insts,
                                                               const int* __restrict__ ids, int jstep,
                                                               const cplx<real>* __restrict__ twg) {
    constexpr int N = 128, L = 32;
    using G = Geo<N>;
    constexpr int M = G::M, P = 4;
    stepper_wave_priority();
    const ColInst<real>& I = insts ? insts[ids[blockIdx.y]] : one;
    if ((I.active && *I.active == 0) || jstep >= I.jmax) return;
    const int lane = threadIdx.x;
    const real* __restrict__ xin = I.xbase + jstep * I.xstride;
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
    const int b = int(blockIdx.x) - 1;
    const int kx = 1 + b / 4, r = b % 4;
    const int q = lane >> 1, c = lane & 1;
    const int m = q < L / 2 ? q : q - L;
    const int jy = P * m + r;
    const bool kp = jy >= -M && jy <= M;
    const int e = kp ? 2 * (jy + M) + c : 0;  // this lane's real number in the column segment
    const double kxv = alpha * kx;
    const double K2 = kxv * kxv + double(jy) * jy;
    const real E1 = kp ? real(exp(-K2 * dt / Re)) : real(0);
    const real Eh = kp ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
    const real g1 = kp ? real(kxv * (1.0 - cprop / K2)) : real(0);
    const real g1s = c ? g1 : -g1;  // i g1 s: real part -g1 Im s, imaginary part g1 Re s
    const real kmask = kp ? real(1.0 / L) : real(0);
    const real nuv = I.negU[bitrev5(q)];  // profile at this lane's grid position after the inverse
    const real* xs = xin + G::seg(kx);
    real w = kp ? xs[e] : real(0);
    real acc = w, s = w;
    SplitTw<real> tw;
    tw.load(twg, q, c);
    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);

    for (int st = 0; st < nsteps; ++st) {
        s = w;
#pragma unroll 4
        for (int stage = 0; stage < 4; ++stage) {
            real v = g1s * xor_lane<1>(s, lane);
            v = split_dif<16>(v, tw, lane);
            v = split_dif<8>(v, tw, lane);
            v = split_dif<4>(v, tw, lane);
            v = split_dif<2>(v, tw, lane);
            v = split_dif<1>(v, tw, lane);
            v *= nuv;
            v = split_dit<1>(v, tw, lane);
            v = split_dit<2>(v, tw, lane);
            v = split_dit<4>(v, tw, lane);
            v = split_dit<8>(v, tw, lane);
            v = split_dit<16>(v, tw, lane);
            const real nh = v * kmask;
            if (stage == 0) {
                acc = E1 * (w + h6 * nh);
                s = Eh * (w + h2 * nh);
            } else if (stage == 1) {
                acc += h3 * Eh * nh;
                s = Eh * w + h2 * nh;
            } else if (stage == 2) {
                acc += h3 * Eh * nh;
                s = E1 * w + hh * Eh * nh;
            } else {
                w = acc + h6 * nh;
            }
        }
    }
    if (kp) yout[G::seg(kx) + e] = w;
}

}  // namespace tsk
