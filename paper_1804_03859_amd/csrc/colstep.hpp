// Column time stepper of the linearized Navier-Stokes operator about a
// parallel base flow (U(y), 0): one 64-lane workgroup owns one dealiased kx
// column for a whole matvec (all T/dt integrating-factor RK4 steps).  The
// design is described with the operator in kolmo.hip.
#pragma once

#include "colfft.hpp"
#include "fft.hpp"

namespace tsk {

template <int N> struct Geo {
    static constexpr int M = (N - 1) / 3;       // largest kept |j|
    static constexpr int NM = 2 * M + 1;        // kept ky per column
    static constexpr int RM = (NM + kWave - 1) / kWave;
    static constexpr int RY = (N + kWave - 1) / kWave;
    static constexpr int64_t n_state = 4ll * M * (M + 1);
    static __host__ __device__ constexpr int64_t seg(int kx) {
        return kx == 0 ? 0 : 2ll * M + int64_t(kx - 1) * 2 * NM;
    }
};

// One operator instance of a (batched) column-stepper launch.  The input of
// step j is xbase + j * xstride (the Arnoldi basis vector v_j; xstride = 0 for a
// plain matvec); `active` (optional) lets finished Arnoldi instances skip.
template <typename real> struct ColInst {
    const real* xbase;
    int64_t xstride;
    real* y;
    const real* negU;
    const real* dOdy;
    double alpha, Re, dt, cprop;
    int nsteps;
    const int* active;
};
struct ColTask {
    int inst;  // index into the instance table
    int kx;    // dealiased column 0..M
};

// ---- the column time stepper ------------------------------------------------------------
// Lane-owned positions: j = lane (< NB = N/RE) and slots r < RE hold the
// y-index / FFT-order wavenumber index pos = j + r NB (colfft.hpp), for the
// spectral state (jy = pos or pos - N, kept when |jy| <= M) and, after the
// inverse transform, for the grid values at y = 2 pi pos / N.
template <typename real, int N, bool PROP>
__global__ __launch_bounds__(kWave) void k_colstep(ColInst<real> one, const ColInst<real>* __restrict__ insts,
                                                   const ColTask* __restrict__ tasks, const cplx<real>* __restrict__ twg,
                                                   int jstep) {
    using C = cplx<real>;
    using G = Geo<N>;
    using PL = ColPlan<N>;
    constexpr int M = G::M, RE = PL::RE, NB = PL::NB;
    static_assert(PL::NBL == 1, "one edge butterfly per lane");
    const ColTask tk = tasks[blockIdx.x];
    const ColInst<real>& I = insts ? insts[tk.inst] : one;
    if (I.active && *I.active == 0) return;
    const real* __restrict__ xin = I.xbase + jstep * I.xstride;
    real* __restrict__ yout = I.y;
    const real* __restrict__ negU = I.negU;
    const real* __restrict__ dOdy = I.dOdy;
    const double alpha = I.alpha, Re = I.Re, dt = I.dt, cprop = I.cprop;
    const int nsteps = I.nsteps;
    const int lane = threadIdx.x;
    const int kx = tk.kx;

    if (kx == 0) {
        // kx = 0: the advection term vanishes identically (d/dx of a y-only
        // field), so the integrating factor alone advances the column.
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

    constexpr int LP = padded_len<N>();
    __shared__ C sA[LP], sB[LP], sT[N];
    __shared__ C sA2[PROP ? 1 : LP], sB2[PROP ? 1 : LP];
    for (int t = lane; t < N; t += kWave) sT[t] = twg[t];

    const double kxv = alpha * kx;
    const bool act = lane < NB;
    real E1[RE], Eh[RE], g1[RE], g2[RE], nu[RE], oy[RE];
    C w[RE], acc[RE], s[RE];
    unsigned keep = 0;
    const real* xs = xin + G::seg(kx);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int pos = lane + r * NB;
        const int jy = pos <= N / 2 ? pos : pos - N;
        const bool kp = act && jy >= -M && jy <= M;
        keep |= kp ? (1u << r) : 0u;
        const double K2 = kxv * kxv + double(jy) * jy;
        E1[r] = kp ? real(exp(-K2 * dt / Re)) : real(0);
        Eh[r] = kp ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
        g1[r] = kp ? (PROP ? real(kxv * (1.0 - cprop / K2)) : real(kxv)) : real(0);
        g2[r] = kp ? real(kxv / K2) : real(0);
        nu[r] = act ? negU[pos] : real(0);
        oy[r] = (!PROP && act) ? dOdy[pos] : real(0);
        const int q = jy + M;
        w[r] = kp ? cmk<C>(xs[2 * q], xs[2 * q + 1]) : cmk<C>(real(0), real(0));
        acc[r] = s[r] = w[r];
    }
    __syncthreads();

    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);
    const real invN = real(1.0 / N);
    C* fwdA = col_result_in_a<N>() ? sB : sA;  // forward transform must not write
    C* fwdB = col_result_in_a<N>() ? sA : sB;  // the buffer the inverse reads last

    for (int st = 0; st < nsteps; ++st) {
#pragma unroll
        for (int r = 0; r < RE; ++r) s[r] = w[r];
#pragma unroll 1
        for (int stage = 0; stage < 4; ++stage) {
            C v[1][RE], v2[1][PROP ? 1 : RE];
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                v[0][r] = cmk<C>(-g1[r] * s[r].y, g1[r] * s[r].x);  // i kx (...) s
                if constexpr (!PROP) v2[0][r] = cmk<C>(-g2[r] * s[r].y, g2[r] * s[r].x);
            }
            col_fft<N, +1>(v, sA, sB, sT, lane);
            if constexpr (!PROP) col_fft<N, +1>(v2, sA2, sB2, sT, lane);
            // product with the base profiles at y = pos
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                C p = cmk<C>(nu[r] * v[0][r].x, nu[r] * v[0][r].y);
                if constexpr (!PROP) {
                    p.x += oy[r] * v2[0][r].x;
                    p.y += oy[r] * v2[0][r].y;
                }
                v[0][r] = p;
            }
            col_fft<N, -1>(v, fwdA, fwdB, sT, lane);
            // Lawson RK4 bookkeeping on the kept modes (registers only)
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                const real kmask = (keep >> r) & 1u ? invN : real(0);
                const C nh = cmk<C>(v[0][r].x * kmask, v[0][r].y * kmask);
                const real e1 = E1[r], eh = Eh[r];
                if (stage == 0) {
                    acc[r] = cmk<C>(e1 * (w[r].x + h6 * nh.x), e1 * (w[r].y + h6 * nh.y));
                    s[r] = cmk<C>(eh * (w[r].x + h2 * nh.x), eh * (w[r].y + h2 * nh.y));
                } else if (stage == 1) {
                    acc[r].x += h3 * eh * nh.x;
                    acc[r].y += h3 * eh * nh.y;
                    s[r] = cmk<C>(eh * w[r].x + h2 * nh.x, eh * w[r].y + h2 * nh.y);
                } else if (stage == 2) {
                    acc[r].x += h3 * eh * nh.x;
                    acc[r].y += h3 * eh * nh.y;
                    s[r] = cmk<C>(e1 * w[r].x + hh * eh * nh.x, e1 * w[r].y + hh * eh * nh.y);
                } else {
                    w[r] = cmk<C>(acc[r].x + h6 * nh.x, acc[r].y + h6 * nh.y);
                }
            }
        }
    }
    real* ys = yout + G::seg(kx);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        if ((keep >> r) & 1u) {
            const int pos = lane + r * NB;
            const int jy = pos <= N / 2 ? pos : pos - N;
            const int q = jy + M;
            ys[2 * q] = w[r].x;
            ys[2 * q + 1] = w[r].y;
        }
    }
}

}  // namespace tsk
