// Column time stepper of the linearized Navier-Stokes operator about a
// parallel base flow (U(y), 0): one 64-lane workgroup owns one dealiased kx
// column for a whole matvec (all T/dt integrating-factor RK4 steps).  The
// design is described with the operator in kolmo.hip.
#pragma once

#include "colfft.hpp"
#include "colxl.hpp"
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

// A time-stepper wave runs for a whole matvec, and the Ritz analyses of earlier
// Arnoldi steps run beside it on other streams; when the dispatcher puts one of
// their waves on the same SIMD, the stepper wave (on the critical path) gets
// the higher issue priority.  Priority only orders instruction issue between
// resident waves: every wave still runs to completion.
__device__ inline void stepper_wave_priority() { __builtin_amdgcn_s_setprio(2); }

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
    // one-harmonic base U = amp sin(nh (y - y0)) (the spectral-coupling stepper of
    // colcouple.hpp): the instance's own cutoff M, the harmonic and its amplitude
    // and phase; unused by the other steppers
    int M, nh;
    double amp, y0;
    // batched restart phase: the instance's input is xbase + jstep xstride while
    // jstep < jmax, later steps skip it (INT_MAX in ordinary runs)
    int jmax;
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
    stepper_wave_priority();
    const ColTask tk = tasks[blockIdx.x];
    const ColInst<real>& I = insts ? insts[tk.inst] : one;
    if ((I.active && *I.active == 0) || jstep >= I.jmax) return;
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

    // N = 128: cross-lane transforms (colxl.hpp), no LDS passes
    constexpr bool kXL = col_xl<N>();
    constexpr int LP = kXL ? 1 : padded_len<N>();
    constexpr int NBUF = kXL ? 1 : COLS * NI;
    __shared__ C sA[NBUF][LP], sB[NBUF][LP], sT[N];
    for (int t = lane; t < N; t += kWave) sT[t] = twg[t];
    static_assert(kWave == 64, "one wavefront per workgroup");
    C* Ai[COLS * NI];
    C* Bi[COLS * NI];
    C* Af[COLS];
    C* Bf[COLS];
#pragma unroll
    for (int c = 0; c < COLS * NI; ++c) {
        Ai[c] = sA[kXL ? 0 : c];
        Bi[c] = sB[kXL ? 0 : c];
    }
    // the forward transform must not write the buffer the inverse reads last
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        Af[c] = col_result_in_a<N>() ? sB[kXL ? 0 : c] : sA[kXL ? 0 : c];
        Bf[c] = col_result_in_a<N>() ? sA[kXL ? 0 : c] : sB[kXL ? 0 : c];
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
        // grid-side profiles at the positions the inverse transform leaves in this slot
        const int gpos = kXL ? xl_grid_pos(lane, r) : pos;
        nu[r] = act ? negU[gpos] : real(0);
        oy[r] = (!PROP && act) ? dOdy[gpos] : real(0);
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
    constexpr bool kTwReg = N <= 256 && !kXL;
    ColTw<N, C> twr;
    if constexpr (kTwReg) twr.load(sT, lane);
    XlTw<C> xtw;
    if constexpr (kXL) xtw.load(sT, lane);

    for (int st = 0; st < nsteps; ++st) {
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int r = 0; r < RE; ++r) s[c][r] = w[c][r];
        // the four stages unrolled: no register moves at the stage switches
#pragma unroll 4
        for (int stage = 0; stage < 4; ++stage) {
            C v[COLS * NI][1][RE];
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    v[c][0][r] = cmk<C>(-g1[c][r] * s[c][r].y, g1[c][r] * s[c][r].x);  // i kx (...) s
                    if constexpr (!PROP) v[COLS + c][0][r] = cmk<C>(-g2[c][r] * s[c][r].y, g2[c][r] * s[c][r].x);
                }
            if constexpr (kXL)
                xl_fft_inv<COLS * NI>(v, xtw, lane);
            else if constexpr (kTwReg)
                col_fft_mr<N, +1, COLS * NI>(v, Ai, Bi, twr, lane);
            else
                col_fft_m<N, +1, COLS * NI>(v, Ai, Bi, sT, lane);
            // product with the base profiles at the grid positions of the slots
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
            if constexpr (kXL)
                xl_fft_fwd<COLS>(pr, xtw, lane);
            else if constexpr (kTwReg)
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

// ---- the transposed column stepper (discrete adjoint) -----------------------------------
// One Lawson step w+ = S w is a polynomial in the diagonal factors E and the
// column advection operator Nc s = (1/N) mask F[nu F^-1(i g1 s) + oy F^-1(i g2 s)]
// (F the forward DFT, F^-1 the unnormalised inverse, g1, g2 zero off the kept
// modes).  In the real Euclidean inner product of the state a complex-linear
// column operator transposes to its conjugate transpose, so
//     Nc^H t = (1/N) [-i g1 F(nu F^-1 t) - i g2 F(oy F^-1 t)]:
// one inverse and one (PROP) or two forward transforms, the products moved to
// the other side of the transforms.  The step transposes stage by stage in
// reverse order (z the adjoint state):
//     s3 = Nc^H(h/6 z),               acc = E1 z + E1 s3
//     s2 = Nc^H(h/3 Eh z + h Eh s3),  acc += Eh s2
//     s1 = Nc^H(h/3 Eh z + h/2 s2),   acc += Eh s1
//     s0 = Nc^H(h/6 E1 z + h/2 Eh s1), z+ = acc + s0.
// M^T is S^T applied T/dt times (the steps are identical).  One column per
// wavefront; the kx = 0 column is diagonal and identical to the forward one.
template <typename real, int N, bool PROP>
__global__ __launch_bounds__(kWave) void k_colstep_adj(ColInst<real> one, const ColTask* __restrict__ tasks,
                                                       const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    using G = Geo<N>;
    using PL = ColPlan<N>;
    constexpr int M = G::M, RE = PL::RE, NB = PL::NB;
    constexpr int NF = PROP ? 1 : 2;  // forward transforms per stage
    static_assert(PL::NBL == 1, "one edge butterfly per lane");
    stepper_wave_priority();
    const ColTask tk = tasks[blockIdx.x];
    const ColInst<real>& I = one;
    const real* __restrict__ xin = I.xbase;
    real* __restrict__ yout = I.y;
    const double alpha = I.alpha, Re = I.Re, dt = I.dt, cprop = I.cprop;
    const int nsteps = I.nsteps;
    const int lane = threadIdx.x;
    const int kx = tk.kx;

    if (kx == 0) {
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

    constexpr bool kXL = col_xl<N>();
    constexpr int LP = kXL ? 1 : padded_len<N>();
    __shared__ C sA[2][LP], sB[2][LP], sT[N];
    for (int t = lane; t < N; t += kWave) sT[t] = twg[t];
    C* Ai[1] = {sA[0]};
    C* Bi[1] = {sB[0]};
    C* Af[NF];
    C* Bf[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) {
        Af[c] = col_result_in_a<N>() ? sB[c] : sA[c];
        Bf[c] = col_result_in_a<N>() ? sA[c] : sB[c];
    }

    const bool act = lane < NB;
    real E1[RE], Eh[RE], g1[RE], g2[RE], nu[RE], oy[RE];
    C z[RE], acc[RE], sprev[RE];
    unsigned keep = 0;
    const double kxv = alpha * kx;
    const real* xs = xin + G::seg(kx);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int pos = lane + r * NB;
        const int jy = pos <= N / 2 ? pos : pos - N;
        const bool kp = act && jy >= -M && jy <= M;
        keep |= kp ? (1u << r) : 0u;
        const int gpos = kXL ? xl_grid_pos(lane, r) : pos;
        nu[r] = act ? I.negU[gpos] : real(0);
        oy[r] = (!PROP && act) ? I.dOdy[gpos] : real(0);
        const double K2 = kxv * kxv + double(jy) * jy;
        E1[r] = kp ? real(exp(-K2 * dt / Re)) : real(0);
        Eh[r] = kp ? real(exp(-K2 * (0.5 * dt) / Re)) : real(0);
        // the 1/N of the forward transform folded into the output factors
        g1[r] = kp ? (PROP ? real(kxv * (1.0 - cprop / K2) / N) : real(kxv / N)) : real(0);
        g2[r] = kp ? real(kxv / K2 / N) : real(0);
        const int q = jy + M;
        z[r] = kp ? cmk<C>(xs[2 * q], xs[2 * q + 1]) : cmk<C>(real(0), real(0));
        acc[r] = sprev[r] = cmk<C>(real(0), real(0));
    }
    __syncthreads();

    const real h6 = real(dt / 6.0), h3 = real(dt / 3.0), h2 = real(0.5 * dt), hh = real(dt);
    constexpr bool kTwReg = N <= 256 && !kXL;
    ColTw<N, C> twr;
    if constexpr (kTwReg) twr.load(sT, lane);
    XlTw<C> xtw;
    if constexpr (kXL) xtw.load(sT, lane);

    for (int st = 0; st < nsteps; ++st) {
#pragma unroll 4
        for (int stage = 0; stage < 4; ++stage) {
            // stage input t (kept modes only)
            C v[1][1][RE];
            if (stage == 0) {
#pragma unroll
                for (int r = 0; r < RE; ++r) v[0][0][r] = cmk<C>(h6 * z[r].x, h6 * z[r].y);
            } else if (stage == 1) {
#pragma unroll
                for (int r = 0; r < RE; ++r)
                    v[0][0][r] = cmk<C>(Eh[r] * (h3 * z[r].x + hh * sprev[r].x), Eh[r] * (h3 * z[r].y + hh * sprev[r].y));
            } else if (stage == 2) {
#pragma unroll
                for (int r = 0; r < RE; ++r)
                    v[0][0][r] = cmk<C>(h3 * Eh[r] * z[r].x + h2 * sprev[r].x, h3 * Eh[r] * z[r].y + h2 * sprev[r].y);
            } else {
#pragma unroll
                for (int r = 0; r < RE; ++r)
                    v[0][0][r] = cmk<C>(h6 * E1[r] * z[r].x + h2 * Eh[r] * sprev[r].x,
                                        h6 * E1[r] * z[r].y + h2 * Eh[r] * sprev[r].y);
            }
            if constexpr (kXL)
                xl_fft_inv<1>(v, xtw, lane);
            else if constexpr (kTwReg)
                col_fft_mr<N, +1, 1>(v, Ai, Bi, twr, lane);
            else
                col_fft_m<N, +1, 1>(v, Ai, Bi, sT, lane);
            C pr[NF][1][RE];
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                pr[0][0][r] = cmk<C>(nu[r] * v[0][0][r].x, nu[r] * v[0][0][r].y);
                if constexpr (!PROP) pr[NF - 1][0][r] = cmk<C>(oy[r] * v[0][0][r].x, oy[r] * v[0][0][r].y);
            }
            if constexpr (kXL)
                xl_fft_fwd<NF>(pr, xtw, lane);
            else if constexpr (kTwReg)
                col_fft_mr<N, -1, NF>(pr, Af, Bf, twr, lane);
            else
                col_fft_m<N, -1, NF>(pr, Af, Bf, sT, lane);
            // s = -i g1 P1 - i g2 P2 (zero off the kept modes)
            C so[RE];
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                C t = cmk<C>(g1[r] * pr[0][0][r].y, -g1[r] * pr[0][0][r].x);
                if constexpr (!PROP) {
                    t.x += g2[r] * pr[NF - 1][0][r].y;
                    t.y -= g2[r] * pr[NF - 1][0][r].x;
                }
                so[r] = t;
            }
            if (stage == 0) {
#pragma unroll
                for (int r = 0; r < RE; ++r)
                    acc[r] = cmk<C>(E1[r] * (z[r].x + so[r].x), E1[r] * (z[r].y + so[r].y));
            } else if (stage == 3) {
#pragma unroll
                for (int r = 0; r < RE; ++r) z[r] = cmk<C>(acc[r].x + so[r].x, acc[r].y + so[r].y);
            } else {
#pragma unroll
                for (int r = 0; r < RE; ++r) {
                    acc[r].x += Eh[r] * so[r].x;
                    acc[r].y += Eh[r] * so[r].y;
                }
            }
#pragma unroll
            for (int r = 0; r < RE; ++r) sprev[r] = so[r];
        }
    }
    real* ys = yout + G::seg(kx);
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        if ((keep >> r) & 1u) {
            const int pos = lane + r * NB;
            const int jy = pos <= N / 2 ? pos : pos - N;
            const int q = jy + M;
            ys[2 * q] = z[r].x;
            ys[2 * q + 1] = z[r].y;
        }
    }
}

}  // namespace tsk
