// Transposed spectral-coupling stepper (discrete adjoint of k_colstep_couple) for
// a parallel base flow of one harmonic, U(y) = amp sin(nh (y - y0)).
//
// Along a chain of modes ky = c + nh t of one kx column the forward advection
// term is N s = D (G s): (N s)_t = G_{t+1} s_{t+1} - G_{t-1} s_{t-1}, with G the
// real factor (amp/2) kx (1 - cprop/K_t^2) (zero beyond the chain) and D the
// difference of the neighbours.  The coefficients are real, so in the real
// Euclidean inner product of the state the transpose is the matrix transpose:
//     (N^T v)_t = G_t (v_{t-1} - v_{t+1}) = -G_t (D v)_t,
// the same neighbour difference, taken of v and scaled afterwards.  The shift of
// the y origin, e^{i ky y0} on input and e^{-i ky y0} on output, is unitary, so
// the transposed propagator keeps it in the same places.  The Lawson RK4 step
// transposes stage by stage in reverse order, as for the column stepper (z the
// adjoint state, s the previous stage's output):
//     s3 = N^T(h/6 z),               acc = E1 z + E1 s3
//     s2 = N^T(h/3 Eh z + h Eh s3),  acc += Eh s2
//     s1 = N^T(h/3 Eh z + h/2 s2),   acc += Eh s1
//     s0 = N^T(h/6 E1 z + h/2 Eh s1), z+ = acc + s0,
// repeated T/dt times.  Launch layout, chain slots and lanes as in the forward
// stepper; the kx = 0 column is diagonal and identical to the forward one.
#pragma once

#include "colcouple.hpp"

namespace tsk {

template <typename real, int S, int WPW>
__global__ __launch_bounds__(kWave * WPW) void k_colstep_couple_adj(ColInst<real> I) {
    static_assert(S == 1 || S == 2, "positions per lane");
    using C = cplx<real>;
    stepper_wave_priority();
    const int M = I.M, nh = I.nh;
    const int slot = int(blockIdx.x) * WPW + (WPW == 1 ? 0 : int(threadIdx.x) / kWave);
    if (slot >= couple_blocks(M, nh)) return;
    const int lane = int(threadIdx.x) % kWave;
    const real* __restrict__ xin = I.xbase;
    real* __restrict__ yout = I.y;
    const double alpha = I.alpha, Re = I.Re, dt = I.dt, cprop = I.cprop;
    const int nsteps = I.nsteps;
    const int NM = 2 * M + 1;
    if (slot == 0) {
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
    const int jy0 = -M + ((c + M) % nh);
    const int len = (M - jy0) / nh + 1;
    const int64_t seg = 2ll * M + int64_t(kx - 1) * 2 * NM;
    const real* xs = xin + seg;
    real* ys = yout + seg;
    bool kp[S];
    int e[S];
    real G[S], E1[S], Eh[S];
    C z[S], acc[S], sp[S], ph[S];
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
        double sn = 0.0, cs = 1.0;
        if (I.y0 != 0.0) sincos(double(jy) * I.y0, &sn, &cs);
        ph[sl] = cmk<C>(real(cs), real(sn));
        const C x = kp[sl] ? cmk<C>(xs[e[sl]], xs[e[sl] + 1]) : cmk<C>(real(0), real(0));
        z[sl] = cmul(x, ph[sl]);
        acc[sl] = sp[sl] = cmk<C>(real(0), real(0));
    }
    // so = N^T v = -G (v_{t+1} - v_{t-1}), v zero beyond the chain
    auto advect_t = [&](const C (&v)[S], C (&so)[S]) {
        C d[S];
        if constexpr (S == 1) {
            d[0].x = wave_move<kDppWaveShl1>(v[0].x) - wave_move<kDppWaveShr1>(v[0].x);
            d[0].y = wave_move<kDppWaveShl1>(v[0].y) - wave_move<kDppWaveShr1>(v[0].y);
        } else {
            // slot 0 holds t = lane, slot 1 t = lane + 64 (as in the forward stepper)
            const bool last = lane == kWave - 1, first = lane == 0;
            const real r0x = wave_move<kDppWaveRol1>(v[0].x), r0y = wave_move<kDppWaveRol1>(v[0].y);
            const real r1x = wave_move<kDppWaveRol1>(v[1].x), r1y = wave_move<kDppWaveRol1>(v[1].y);
            const real l0x = wave_move<kDppWaveRor1>(v[0].x), l0y = wave_move<kDppWaveRor1>(v[0].y);
            const real l1x = wave_move<kDppWaveRor1>(v[1].x), l1y = wave_move<kDppWaveRor1>(v[1].y);
            d[0].x = (last ? r1x : r0x) - (first ? real(0) : l0x);
            d[0].y = (last ? r1y : r0y) - (first ? real(0) : l0y);
            d[1].x = (last ? real(0) : r1x) - (first ? l0x : l1x);
            d[1].y = (last ? real(0) : r1y) - (first ? l0y : l1y);
        }
#pragma unroll
        for (int sl = 0; sl < S; ++sl) so[sl] = cmk<C>(-G[sl] * d[sl].x, -G[sl] * d[sl].y);
    };
    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);
    for (int st = 0; st < nsteps; ++st) {
        C v[S], so[S];
        // stage 3 of the forward step first: s3 = N^T(h/6 z), acc = E1 (z + s3)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) v[sl] = cmk<C>(h6 * z[sl].x, h6 * z[sl].y);
        advect_t(v, so);
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(E1[sl] * (z[sl].x + so[sl].x), E1[sl] * (z[sl].y + so[sl].y));
            sp[sl] = so[sl];
        }
        // s2 = N^T(Eh (h/3 z + h s3)), acc += Eh s2
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
            v[sl] = cmk<C>(Eh[sl] * fma(hh, sp[sl].x, h3 * z[sl].x), Eh[sl] * fma(hh, sp[sl].y, h3 * z[sl].y));
        advect_t(v, so);
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(fma(Eh[sl], so[sl].x, acc[sl].x), fma(Eh[sl], so[sl].y, acc[sl].y));
            sp[sl] = so[sl];
        }
        // s1 = N^T(h/3 Eh z + h/2 s2), acc += Eh s1
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
            v[sl] = cmk<C>(fma(h2, sp[sl].x, h3 * Eh[sl] * z[sl].x), fma(h2, sp[sl].y, h3 * Eh[sl] * z[sl].y));
        advect_t(v, so);
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            acc[sl] = cmk<C>(fma(Eh[sl], so[sl].x, acc[sl].x), fma(Eh[sl], so[sl].y, acc[sl].y));
            sp[sl] = so[sl];
        }
        // s0 = N^T(h/6 E1 z + h/2 Eh s1), z+ = acc + s0
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
            v[sl] = cmk<C>(fma(h2 * Eh[sl], sp[sl].x, h6 * E1[sl] * z[sl].x),
                           fma(h2 * Eh[sl], sp[sl].y, h6 * E1[sl] * z[sl].y));
        advect_t(v, so);
#pragma unroll
        for (int sl = 0; sl < S; ++sl) z[sl] = cmk<C>(acc[sl].x + so[sl].x, acc[sl].y + so[sl].y);
    }
#pragma unroll
    for (int sl = 0; sl < S; ++sl)
        if (kp[sl]) {
            const C out = cmulc(ph[sl], z[sl]);  // e^{-i ky y0} z
            ys[e[sl]] = out.x;
            ys[e[sl] + 1] = out.y;
        }
}

}  // namespace tsk
