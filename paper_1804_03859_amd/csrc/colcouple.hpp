// Spectral-coupling time stepper for a parallel base flow of one harmonic,
// U(y) = amp sin(nh (y - y0)) with dOmega/dy = cprop U (the Kolmogorov flow
// sin 4y: nh = 4, cprop = 16, y0 = 0).
//
// The linearized vorticity equation about U (Sec. 3, eq. "linearized
// Navier-Stokes equations", vorticity form) has the advection term
//     N(omega) = -(U d_x omega + v dOmega/dy) = -U d_x (omega - cprop psi),
// psi^ = omega^ / K^2.  In the kx column, with f^ = i kx (1 - cprop/K^2) omega^,
// the product with one harmonic couples ky only to ky +- nh:
//     N^(ky) = -(U f)^(ky) = (i amp / 2) (f^(ky - nh) - f^(ky + nh))  (y0 = 0).
// With the 2/3 rule (|ky| <= M) and nh < N - 2M no term of the pseudo-spectral
// product on the N-point grid wraps onto a kept mode, so this three-point
// coupling equals the pseudo-spectral product with the mask applied, to
// rounding; the transforms around the product cancel exactly.  A phase y0 is
// a shift of the y origin: the state is multiplied by e^{i ky y0} on input and
// by e^{-i ky y0} on output, and the stepper runs with y0 = 0.
//
// The modes of a column split into nh chains ky = c + nh t (c the residue of ky
// mod nh), each coupled only along itself.  Writing q_t = (amp/2) kx (1 -
// cprop/K_t^2) s_t (a real factor times the complex mode), the advection term
// of chain position t is N_t = q_{t+1} - q_{t-1}, with q = 0 beyond the chain's
// kept range.  One wavefront advances one chain for the whole matvec (all T/dt
// Lawson RK4 steps, state in registers): lane l holds position t = l (and t =
// l + 64 when the chain is longer than 64), and the neighbours come from DPP
// whole-wavefront shifts (lane l reads lane l + 1 or l - 1; the end lanes read
// zero, or the other slot's end value through the rotations when S = 2).
// Positions beyond the chain have a zero factor, so they never feed back.
#pragma once

#include "colstep.hpp"

namespace tsk {

// Whole-wavefront DPP moves of a 32-bit word: SHL lane l <- l + 1 (lane 63 <- 0),
// SHR lane l <- l - 1 (lane 0 <- 0), ROL lane l <- (l + 1) mod 64, ROR lane l <-
// (l - 1) mod 64.
enum : int { kDppWaveShl1 = 0x130, kDppWaveRol1 = 0x134, kDppWaveShr1 = 0x138, kDppWaveRor1 = 0x13C };
template <int CTRL> __device__ inline float wave_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ inline double wave_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Workgroups of a coupling launch for one instance: the kx = 0 column, then the
// nh chains of every column kx = 1..M.
__host__ __device__ inline int couple_blocks(int M, int nh) { return 1 + nh * M; }

// Wavefront w of the grid (w = blockIdx.x WPW + wave in the workgroup) takes
// chain slot w: at least couple_blocks(M, nh) of the largest instance (slots
// beyond an instance's own count return at once).  WPW: wavefronts per
// workgroup (the launch shape the library tunes; every wavefront computes its
// chain alone, so the results do not depend on it).  Grid y: the instance,
// insts[ids[y]] of a batch (input of Arnoldi step jstep: xbase + jstep xstride;
// finished instances skip), or `one` when insts is null.  S: positions per lane
// (chains of up to 64 S modes).  Lawson RK4 as the other column steppers.
template <typename real, int S, int WPW>
__global__ __launch_bounds__(kWave * WPW) void k_colstep_couple(ColInst<real> one,
                                                                const ColInst<real>* __restrict__ insts,
                                                                const int* __restrict__ ids, int jstep) {
    static_assert(S == 1 || S == 2, "positions per lane");
    using C = cplx<real>;
    stepper_wave_priority();
    const ColInst<real>& I = insts ? insts[ids[blockIdx.y]] : one;
    if ((I.active && *I.active == 0) || jstep >= I.jmax) return;
    const int M = I.M, nh = I.nh;
    const int slot = int(blockIdx.x) * WPW + (WPW == 1 ? 0 : int(threadIdx.x) / kWave);
    if (slot >= couple_blocks(M, nh)) return;
    const int lane = int(threadIdx.x) % kWave;
    const real* __restrict__ xin = I.xbase + jstep * I.xstride;
    real* __restrict__ yout = I.y;
    const double alpha = I.alpha, Re = I.Re, dt = I.dt, cprop = I.cprop;
    const int nsteps = I.nsteps;
    const int NM = 2 * M + 1;
    if (slot == 0) {
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
    const int b = slot - 1;
    const int kx = 1 + b / nh, c = b % nh;
    const double kxv = alpha * kx;
    // first kept ky of the chain (ky = c mod nh) and its length
    const int jy0 = -M + ((c + M) % nh);
    const int len = (M - jy0) / nh + 1;
    const int64_t seg = 2ll * M + int64_t(kx - 1) * 2 * NM;
    const real* xs = xin + seg;
    real* ys = yout + seg;
    bool kp[S];
    int e[S];
    real G[S], E1[S], Eh[S], E1h6[S], Ehh2[S], h3Eh[S], hhEh[S];
    C w[S], acc[S], sv[S], ph[S];
    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
        const int t = lane + kWave * sl;
        kp[sl] = t < len;
        const int jy = jy0 + nh * (kp[sl] ? t : 0);
        e[sl] = 2 * (jy + M);
        const double K2 = kxv * kxv + double(jy) * jy;
        G[sl] = kp[sl] ? real(0.5 * I.amp * kxv * (1.0 - cprop / K2)) : real(0);
        E1[sl] = kp[sl] ? real(exp(-K2 * dt / Re)) : real(0);
        Eh[sl] = kp[sl] ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
        E1h6[sl] = E1[sl] * h6;
        Ehh2[sl] = Eh[sl] * h2;
        h3Eh[sl] = h3 * Eh[sl];
        hhEh[sl] = hh * Eh[sl];
        // e^{i ky y0}: the shift of the y origin that makes the profile amp sin(nh y)
        double sn = 0.0, cs = 1.0;
        if (I.y0 != 0.0) sincos(double(jy) * I.y0, &sn, &cs);
        ph[sl] = cmk<C>(real(cs), real(sn));
        const C x = kp[sl] ? cmk<C>(xs[e[sl]], xs[e[sl] + 1]) : cmk<C>(real(0), real(0));
        w[sl] = cmul(x, ph[sl]);
        acc[sl] = sv[sl] = w[sl];
    }
    // advection term of the current stage input sv: nh_t = q_{t+1} - q_{t-1}
    auto advect = [&](C (&nt)[S]) {
        C q[S];
#pragma unroll
        for (int sl = 0; sl < S; ++sl) q[sl] = cmk<C>(G[sl] * sv[sl].x, G[sl] * sv[sl].y);
        if constexpr (S == 1) {
            nt[0].x = wave_move<kDppWaveShl1>(q[0].x) - wave_move<kDppWaveShr1>(q[0].x);
            nt[0].y = wave_move<kDppWaveShl1>(q[0].y) - wave_move<kDppWaveShr1>(q[0].y);
        } else {
            // slot 0 holds t = lane, slot 1 t = lane + 64: the right neighbour of
            // lane 63 in slot 0 is lane 0 of slot 1, the left neighbour of lane 0
            // in slot 1 is lane 63 of slot 0
            const bool last = lane == kWave - 1, first = lane == 0;
            const real r0x = wave_move<kDppWaveRol1>(q[0].x), r0y = wave_move<kDppWaveRol1>(q[0].y);
            const real r1x = wave_move<kDppWaveRol1>(q[1].x), r1y = wave_move<kDppWaveRol1>(q[1].y);
            const real l0x = wave_move<kDppWaveRor1>(q[0].x), l0y = wave_move<kDppWaveRor1>(q[0].y);
            const real l1x = wave_move<kDppWaveRor1>(q[1].x), l1y = wave_move<kDppWaveRor1>(q[1].y);
            nt[0].x = (last ? r1x : r0x) - (first ? real(0) : l0x);
            nt[0].y = (last ? r1y : r0y) - (first ? real(0) : l0y);
            nt[1].x = (last ? real(0) : r1x) - (first ? l0x : l1x);
            nt[1].y = (last ? real(0) : r1y) - (first ? l0y : l1y);
        }
    };
    for (int st = 0; st < nsteps; ++st) {
        C E1w[S], Ehw[S];
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            E1w[sl] = cmk<C>(E1[sl] * w[sl].x, E1[sl] * w[sl].y);
            Ehw[sl] = cmk<C>(Eh[sl] * w[sl].x, Eh[sl] * w[sl].y);
            sv[sl] = w[sl];
        }
        C nt[S];
        advect(nt);  // stage 1: a = N(w)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(fma(E1h6[sl], nt[sl].x, E1w[sl].x), fma(E1h6[sl], nt[sl].y, E1w[sl].y));
            sv[sl] = cmk<C>(fma(Ehh2[sl], nt[sl].x, Ehw[sl].x), fma(Ehh2[sl], nt[sl].y, Ehw[sl].y));
        }
        advect(nt);  // stage 2: b = N(E_h (w + h/2 a))
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(fma(h3Eh[sl], nt[sl].x, acc[sl].x), fma(h3Eh[sl], nt[sl].y, acc[sl].y));
            sv[sl] = cmk<C>(fma(h2, nt[sl].x, Ehw[sl].x), fma(h2, nt[sl].y, Ehw[sl].y));
        }
        advect(nt);  // stage 3: c = N(E_h w + h/2 b)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(fma(h3Eh[sl], nt[sl].x, acc[sl].x), fma(h3Eh[sl], nt[sl].y, acc[sl].y));
            sv[sl] = cmk<C>(fma(hhEh[sl], nt[sl].x, E1w[sl].x), fma(hhEh[sl], nt[sl].y, E1w[sl].y));
        }
        advect(nt);  // stage 4: d = N(E_1 w + h E_h c)
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
            w[sl] = cmk<C>(fma(h6, nt[sl].x, acc[sl].x), fma(h6, nt[sl].y, acc[sl].y));
    }
#pragma unroll
    for (int sl = 0; sl < S; ++sl)
        if (kp[sl]) {
            const C out = cmulc(ph[sl], w[sl]);  // e^{-i ky y0} w
            ys[e[sl]] = out.x;
            ys[e[sl] + 1] = out.y;
        }
}

}  // namespace tsk
