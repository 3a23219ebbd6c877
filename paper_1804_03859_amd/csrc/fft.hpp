// Workgroup-local complex FFT of compile-time length N = 2^a 3^b held in LDS.
//
// Stockham auto-sort formulation: pass p with radix R reads the R inputs of
// butterfly j at stride N/R, applies the twiddles W_{Ns R}^{(j mod Ns) r},
// transforms them with an in-register R-point DFT and writes them at
// (j / Ns) Ns R + (j mod Ns) + r Ns, where Ns is the product of the radices of
// the earlier passes.  After the last pass the data are in natural order, so no
// bit reversal is needed.  Radices 8, 4, 2 and 3 (3 for the 384-point grid).
//
// The twiddle table tw[t] = exp(-2 pi i t / N) lives in LDS; the inverse
// transform (SIGN = +1, unnormalised) uses its conjugate.  Every pass ends with
// a workgroup barrier; the caller owns the two N-element ping-pong buffers.
#pragma once

#include "common.hpp"

namespace tsk {

// ---- radix plan --------------------------------------------------------------
constexpr int fft_num_passes(int N) {
    int p = 0;
    while (N % 8 == 0 && N > 1) { N /= 8; ++p; }
    while (N % 4 == 0 && N > 1) { N /= 4; ++p; }
    while (N % 2 == 0 && N > 1) { N /= 2; ++p; }
    while (N % 3 == 0 && N > 1) { N /= 3; ++p; }
    return p;
}
constexpr int fft_radix(int N, int pass) {
    int p = 0;
    while (N % 8 == 0 && N > 1) { if (p == pass) return 8; N /= 8; ++p; }
    while (N % 4 == 0 && N > 1) { if (p == pass) return 4; N /= 4; ++p; }
    while (N % 2 == 0 && N > 1) { if (p == pass) return 2; N /= 2; ++p; }
    while (N % 3 == 0 && N > 1) { if (p == pass) return 3; N /= 3; ++p; }
    return 1;
}
constexpr bool fft_supported(int N) {
    if (N < 2) return false;
    while (N % 2 == 0) N /= 2;
    while (N % 3 == 0) N /= 3;
    return N == 1;
}

// ---- small DFTs in registers ---------------------------------------------------
// Multiply by (SIGN * i): SIGN = -1 gives -i (forward), +1 gives +i (inverse).
template <int SIGN, typename C> __device__ inline C mul_si(C a) {
    if constexpr (SIGN < 0) return cmk<C>(a.y, -a.x);
    else return cmk<C>(-a.y, a.x);
}

template <int SIGN, typename C> __device__ inline void dft2(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int SIGN, typename C> __device__ inline void dft4(C* v) {
    C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    C b0 = cadd(v[1], v[3]), b1 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
}

template <int SIGN, typename C> __device__ inline void dft8(C* v) {
    using R = decltype(C{}.x);
    const R h = R(0.70710678118654752440084436210485);
    // split into even / odd 4-point DFTs
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    dft4<SIGN>(e);
    dft4<SIGN>(o);
    // twiddles W8^{SIGN*q} for q = 1, 2, 3 (W8 = exp(2 pi i / 8))
    C o1 = o[1], o2 = o[2], o3 = o[3];
    if constexpr (SIGN < 0) {
        o1 = cmk<C>(h * (o1.x + o1.y), h * (o1.y - o1.x));
        o2 = cmk<C>(o2.y, -o2.x);
        o3 = cmk<C>(h * (-o3.x + o3.y), h * (-o3.y - o3.x));
    } else {
        o1 = cmk<C>(h * (o1.x - o1.y), h * (o1.y + o1.x));
        o2 = cmk<C>(-o2.y, o2.x);
        o3 = cmk<C>(h * (-o3.x - o3.y), h * (-o3.y + o3.x));
    }
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int SIGN, typename C> __device__ inline void dft3(C* v) {
    using R = decltype(C{}.x);
    const R c = R(-0.5);
    const R s = R(SIGN) * R(0.86602540378443864676372317075294);
    C t = cadd(v[1], v[2]);
    C d = csub(v[1], v[2]);
    C m = cmk<C>(v[0].x + c * t.x, v[0].y + c * t.y);
    // (SIGN i sqrt3/2) * d
    C r = cmk<C>(-s * d.y, s * d.x);
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <int R, int SIGN, typename C> __device__ inline void dft(C* v) {
    if constexpr (R == 2) dft2<SIGN>(v);
    else if constexpr (R == 3) dft3<SIGN>(v);
    else if constexpr (R == 4) dft4<SIGN>(v);
    else dft8<SIGN>(v);
}

// ---- one Stockham pass ----------------------------------------------------------
template <int N, int R, int NS, int SIGN, int NT, typename C>
__device__ inline void fft_pass(const C* __restrict__ in, C* __restrict__ out, const C* __restrict__ tw, int tid) {
    constexpr int NB = N / R;          // butterflies
    constexpr int TS = N / (NS * R);   // twiddle stride in the table
    for (int j = tid; j < NB; j += NT) {
        const int k = j % NS;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C x = in[j + r * NB];
            if (NS > 1 && r > 0) {
                C w = tw[k * r * TS];
                if constexpr (SIGN > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            v[r] = x;
        }
        dft<R, SIGN>(v);
        const int o = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[o + r * NS] = v[r];
    }
}

template <int N, int P, int NS, int SIGN, int NT, typename C>
__device__ inline C* fft_passes(C* a, C* b, const C* tw, int tid) {
    if constexpr (P >= fft_num_passes(N)) {
        return a;
    } else {
        constexpr int R = fft_radix(N, P);
        fft_pass<N, R, NS, SIGN, NT>(a, b, tw, tid);
        __syncthreads();
        return fft_passes<N, P + 1, NS * R, SIGN, NT>(b, a, tw, tid);
    }
}

// Transform the N values in `a` (LDS); `b` is scratch.  Returns the buffer that
// holds the result (a or b).  Caller must have synchronised `a` and `tw`.
template <int N, int SIGN, int NT, typename C>
__device__ inline C* fft_lds(C* a, C* b, const C* tw, int tid) {
    return fft_passes<N, 0, 1, SIGN, NT>(a, b, tw, tid);
}

}  // namespace tsk
