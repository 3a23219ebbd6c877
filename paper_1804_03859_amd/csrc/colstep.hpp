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
    int kx;    // first dealiased column 0..M
    int ncol;  // columns kx .. kx + ncol - 1 (kx = 0 only alone)
};

// ---- the column time stepper ------------------------------------------------------------
// Lane-owned positions: j = lane (< NB = N/RE) and slots r < RE hold the
// y-index / FFT-order wavenumber index pos = j + r NB (colfft.hpp), for the
// spectral state (jy = pos or pos - N, kept when |jy| <= M) and, after the
// inverse transform, for the grid values at y = 2 pi pos / N.  A workgroup
// advances COLS columns of one instance at once (their transforms interleaved,
// see col_fft_m); a task with fewer columns computes zeros for the rest.
template <typename real, int N, bool PROP, int COLS>
__global__ __launch_bounds__(kWave) void k_colstep(ColInst<real> one, const ColInst<real>* __restrict__ insts,
                                                   const ColTask* __restrict__ tasks, const cplx<real>* __restrict__ twg,
                                                   int jstep) {
    using C = cplx<real>;
    using G = Geo<N>;
    using PL = ColPlan<N>;
    constexpr int M = G::M, RE = PL::RE, NB = PL::NB;
    constexpr int NI = PROP ? 1 : 2;  // inverse transforms per column and stage
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
    const int kx0 = tk.kx, ncol = tk.ncol;

    if (kx0 == 0) {
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
    __shared__ C sA[COLS * NI][LP], sB[COLS * NI][LP], sT[N];
    for (int t = lane; t < N; t += kWave) sT[t] = twg[t];
    static_assert(kWave == 64, "one wavefront per workgroup");
    C* Ai[COLS * NI];
    C* Bi[COLS * NI];
    C* Af[COLS];
    C* Bf[COLS];
#pragma unroll
    for (int c = 0; c < COLS * NI; ++c) {
        Ai[c] = sA[c];
        Bi[c] = sB[c];
    }
    // the forward transform must not write the buffer the inverse reads last
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        Af[c] = col_result_in_a<N>() ? sB[c] : sA[c];
        Bf[c] = col_result_in_a<N>() ? sA[c] : sB[c];
    }

    const bool act = lane < NB;
    real E1[COLS][RE], Eh[COLS][RE], g1[COLS][RE], g2[COLS][RE], nu[RE], oy[RE];
    C w[COLS][RE], acc[COLS][RE], s[COLS][RE];
    unsigned keep = 0;
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int pos = lane + r * NB;
        const int jy = pos <= N / 2 ? pos : pos - N;
        const bool kp = act && jy >= -M && jy <= M;
        keep |= kp ? (1u << r) : 0u;
        nu[r] = act ? negU[pos] : real(0);
        oy[r] = (!PROP && act) ? dOdy[pos] : real(0);
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            const bool kc = kp && c < ncol;
            const int kx = kx0 + c;
            const double kxv = alpha * kx;
            const double K2 = kxv * kxv + double(jy) * jy;
            E1[c][r] = kc ? real(exp(-K2 * dt / Re)) : real(0);
            Eh[c][r] = kc ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
            g1[c][r] = kc ? (PROP ? real(kxv * (1.0 - cprop / K2)) : real(kxv)) : real(0);
            g2[c][r] = kc ? real(kxv / K2) : real(0);
            const int q = jy + M;
            const real* xs = xin + G::seg(kx);
            w[c][r] = kc ? cmk<C>(xs[2 * q], xs[2 * q + 1]) : cmk<C>(real(0), real(0));
            acc[c][r] = s[c][r] = w[c][r];
        }
    }
    __syncthreads();

    const real hh = real(dt), h2 = real(0.5 * dt), h3 = real(dt / 3.0), h6 = real(dt / 6.0);
    const real invN = real(1.0 / N);
    // twiddles in registers where the register budget allows (N <= 256)
    constexpr bool kTwReg = N <= 256;
    ColTw<N, C> twr;
    if constexpr (kTwReg) twr.load(sT, lane);

    for (int st = 0; st < nsteps; ++st) {
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int r = 0; r < RE; ++r) s[c][r] = w[c][r];
#pragma unroll 1
        for (int stage = 0; stage < 4; ++stage) {
            C v[COLS * NI][1][RE];
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    v[c][0][r] = cmk<C>(-g1[c][r] * s[c][r].y, g1[c][r] * s[c][r].x);  // i kx (...) s
                    if constexpr (!PROP) v[COLS + c][0][r] = cmk<C>(-g2[c][r] * s[c][r].y, g2[c][r] * s[c][r].x);
                }
            if constexpr (kTwReg)
                col_fft_mr<N, +1, COLS * NI>(v, Ai, Bi, twr, lane);
            else
                col_fft_m<N, +1, COLS * NI>(v, Ai, Bi, sT, lane);
            // product with the base profiles at y = pos
            C pr[COLS][1][RE];
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    C p = cmk<C>(nu[r] * v[c][0][r].x, nu[r] * v[c][0][r].y);
                    if constexpr (!PROP) {
                        p.x += oy[r] * v[COLS + c][0][r].x;
                        p.y += oy[r] * v[COLS + c][0][r].y;
                    }
                    pr[c][0][r] = p;
                }
            if constexpr (kTwReg)
                col_fft_mr<N, -1, COLS>(pr, Af, Bf, twr, lane);
            else
                col_fft_m<N, -1, COLS>(pr, Af, Bf, sT, lane);
            // Lawson RK4 bookkeeping on the kept modes (registers only); the stage
            // switch is outside the column/slot loops so it stays a uniform branch
            C nh[COLS][RE];
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    const real kmask = (keep >> r) & 1u ? invN : real(0);
                    nh[c][r] = cmk<C>(pr[c][0][r].x * kmask, pr[c][0][r].y * kmask);
                }
            if (stage == 0) {
#pragma unroll
                for (int c = 0; c < COLS; ++c)
#pragma unroll
                    for (int r = 0; r < RE; ++r) {
                        const real e1 = E1[c][r], eh = Eh[c][r];
                        acc[c][r] = cmk<C>(e1 * (w[c][r].x + h6 * nh[c][r].x), e1 * (w[c][r].y + h6 * nh[c][r].y));
                        s[c][r] = cmk<C>(eh * (w[c][r].x + h2 * nh[c][r].x), eh * (w[c][r].y + h2 * nh[c][r].y));
                    }
            } else if (stage == 1) {
#pragma unroll
                for (int c = 0; c < COLS; ++c)
#pragma unroll
                    for (int r = 0; r < RE; ++r) {
                        const real eh = Eh[c][r];
                        acc[c][r].x += h3 * eh * nh[c][r].x;
                        acc[c][r].y += h3 * eh * nh[c][r].y;
                        s[c][r] = cmk<C>(eh * w[c][r].x + h2 * nh[c][r].x, eh * w[c][r].y + h2 * nh[c][r].y);
                    }
            } else if (stage == 2) {
#pragma unroll
                for (int c = 0; c < COLS; ++c)
#pragma unroll
                    for (int r = 0; r < RE; ++r) {
                        const real e1 = E1[c][r], eh = Eh[c][r];
                        acc[c][r].x += h3 * eh * nh[c][r].x;
                        acc[c][r].y += h3 * eh * nh[c][r].y;
                        s[c][r] = cmk<C>(e1 * w[c][r].x + hh * eh * nh[c][r].x, e1 * w[c][r].y + hh * eh * nh[c][r].y);
                    }
            } else {
#pragma unroll
                for (int c = 0; c < COLS; ++c)
#pragma unroll
                    for (int r = 0; r < RE; ++r)
                        w[c][r] = cmk<C>(acc[c][r].x + h6 * nh[c][r].x, acc[c][r].y + h6 * nh[c][r].y);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        if (c >= ncol) continue;
        real* ys = yout + G::seg(kx0 + c);
#pragma unroll
        for (int r = 0; r < RE; ++r) {
            if ((keep >> r) & 1u) {
                const int pos = lane + r * NB;
                const int jy = pos <= N / 2 ? pos : pos - N;
                const int q = jy + M;
                ys[2 * q] = w[c][r].x;
                ys[2 * q + 1] = w[c][r].y;
            }
        }
    }
}

}  // namespace tsk
