// Single-wavefront complex FFT of length N whose first and last passes work
// on registers, for the column time stepper.
//
// Plan: N = RE * (middle radices) * RE with the same "edge" radix RE for the
// first and the last Stockham pass.  Lane-owned butterfly j
// (0 <= j < NB = N/RE) of the first pass reads positions j + r NB; the last
// pass of the same plan writes its butterfly j to exactly those positions.  So a
// lane that keeps the data of "its" positions in registers can (i) feed the first
// pass without an LDS read, (ii) take the last pass's outputs without an LDS
// write, and (iii) chain an inverse transform, a pointwise product and a
// forward transform with LDS traffic only inside each transform
// (1 + number-of-middle-passes round trips per transform).
//
// LDS buffers use a padded index pad(i) = i + i/8, which spreads the stride-R
// writes of the first pass over all banks.
#pragma once

#include "fft.hpp"

namespace tsk {

__host__ __device__ constexpr int pad8(int i) { return i + (i >> 3); }
template <int N> constexpr int padded_len() { return N + N / 8 + 1; }

// Edge radix: the smallest that leaves at most one edge butterfly per lane
// (N / RE <= 64) and an integral middle length N / RE^2, so that every lane
// owns RE positions and all 64 lanes work in the edge passes when N >= 128.
constexpr int col_edge_radix(int N) {
    for (int r : {2, 4, 8, 3})
        if (N % (r * r) == 0 && N / r <= kWave) return r;
    return 8;
}
// Middle radices: 8 only when its butterflies still fill the wavefront
// (N / 8 >= 64), otherwise 4, then 2, then 3 (fewer idle lanes per pass).
constexpr int col_mid_radix(int N, int mid, int pass) {
    int p = 0;
    while (mid > 1) {
        int r = (mid % 8 == 0 && N / 8 >= kWave) ? 8 : (mid % 4 == 0) ? 4 : (mid % 2 == 0) ? 2 : 3;
        if (p == pass) return r;
        mid /= r;
        ++p;
    }
    return 1;
}
constexpr int col_mid_passes(int N, int mid) {
    int p = 0;
    while (col_mid_radix(N, mid, p) > 1) ++p;
    return p;
}

template <int N> struct ColPlan {
    static constexpr int RE = col_edge_radix(N);
    static constexpr int MID = N / (RE * RE);
    static constexpr int NMID = col_mid_passes(N, MID);
    static constexpr int NB = N / RE;                     // butterflies of an edge pass
    static constexpr int NBL = (NB + kWave - 1) / kWave;  // per lane
    static_assert(RE * RE * MID == N, "unsupported length");
};

// One middle Stockham pass (LDS -> LDS, padded), radix R, stride NS.
template <int N, int R, int NS, int SIGN, typename C>
__device__ inline void col_mid_pass(const C* __restrict__ in, C* __restrict__ out, const C* __restrict__ tw,
                                    int lane) {
    constexpr int NB = N / R;
    constexpr int TS = N / (NS * R);
    for (int j = lane; j < NB; j += kWave) {
        const int k = j % NS;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C x = in[pad8(j + r * NB)];
            if (r > 0) {
                C w = tw[k * r * TS];
                if constexpr (SIGN > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            v[r] = x;
        }
        dft<R, SIGN>(v);
        const int o = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[pad8(o + r * NS)] = v[r];
    }
}

template <int N, int P, int NS, int SIGN, typename C>
__device__ inline C* col_mid_passes(C* a, C* b, const C* tw, int lane) {
    using PL = ColPlan<N>;
    if constexpr (P >= PL::NMID) {
        return a;
    } else {
        constexpr int R = col_mid_radix(N, PL::MID, P);
        col_mid_pass<N, R, NS, SIGN>(a, b, tw, lane);
        __syncthreads();
        return col_mid_passes<N, P + 1, NS * R, SIGN>(b, a, tw, lane);
    }
}

// Whole transform: v[b][r] holds position j + r NB (j = lane + 64 b) on entry
// and on exit.  The first pass writes `a`; returns nothing (result in v).
// Uses a and b as LDS scratch.
template <int N, int SIGN, typename C>
__device__ inline void col_fft(C (&v)[ColPlan<N>::NBL][ColPlan<N>::RE], C* a, C* b, const C* tw, int lane) {
    using PL = ColPlan<N>;
    constexpr int RE = PL::RE, NB = PL::NB;
    // first pass (stride 1, no twiddles) from registers
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
            dft<RE, SIGN>(v[q]);
#pragma unroll
            for (int r = 0; r < RE; ++r) a[pad8(j * RE + r)] = v[q][r];
        }
    }
    __syncthreads();
    const C* src = col_mid_passes<N, 0, RE, SIGN>(a, b, tw, lane);
    // last pass (stride NB) into registers
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
#pragma unroll
            for (int r = 0; r < RE; ++r) {
                C x = src[pad8(j + r * NB)];
                if (r > 0) {
                    C w = tw[j * r];
                    if constexpr (SIGN > 0) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[q][r] = x;
            }
            dft<RE, SIGN>(v[q]);
        }
    }
}

// ---- several independent columns per wavefront ----------------------------------
// The same transform on COLS columns at once, for a workgroup of one
// wavefront (passes are separated by wave_lds_sync, not workgroup barriers).
// Every pass first loads the butterfly inputs of all columns, then computes,
// then stores, so the LDS
// latency of one column overlaps the arithmetic of the others (a lone
// wavefront per SIMD has no other way to hide it).  Each column has its own
// pair of LDS buffers; twiddles are shared.
template <int N, int R, int NS, int SIGN, int COLS, typename C>
__device__ inline void col_mid_pass_m(C* const* in, C* const* out, const C* __restrict__ tw, int lane) {
    constexpr int NB = N / R;
    constexpr int TS = N / (NS * R);
    for (int j = lane; j < NB; j += kWave) {
        const int k = j % NS;
        C w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            w[r] = tw[k * r * TS];
            if constexpr (SIGN > 0) w[r].y = -w[r].y;
        }
        C v[COLS][R];
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) v[c][r] = in[c][pad8(j + r * NB)];
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], w[r]);
            dft<R, SIGN>(v[c]);
        }
        const int o = (j / NS) * NS * R + k;
#pragma unroll
        for (int c = 0; c < COLS; ++c)
#pragma unroll
            for (int r = 0; r < R; ++r) out[c][pad8(o + r * NS)] = v[c][r];
    }
}

template <int N, int P, int NS, int SIGN, int COLS, typename C>
__device__ inline bool col_mid_passes_m(C* const* a, C* const* b, const C* tw, int lane) {
    using PL = ColPlan<N>;
    if constexpr (P >= PL::NMID) {
        return true;  // result in a
    } else {
        constexpr int R = col_mid_radix(N, PL::MID, P);
        col_mid_pass_m<N, R, NS, SIGN, COLS>(a, b, tw, lane);
        wave_lds_sync();
        return !col_mid_passes_m<N, P + 1, NS * R, SIGN, COLS>(b, a, tw, lane);
    }
}

// v[c][b][r] holds position j + r NB of column c (j = lane + 64 b) on entry and
// on exit.  a[c], b[c]: LDS buffers of column c.
template <int N, int SIGN, int COLS, typename C>
__device__ inline void col_fft_m(C (&v)[COLS][ColPlan<N>::NBL][ColPlan<N>::RE], C* const* a, C* const* b,
                                 const C* tw, int lane) {
    using PL = ColPlan<N>;
    constexpr int RE = PL::RE, NB = PL::NB;
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                dft<RE, SIGN>(v[c][q]);
#pragma unroll
                for (int r = 0; r < RE; ++r) a[c][pad8(j * RE + r)] = v[c][q][r];
            }
        }
    }
    wave_lds_sync();
    const bool in_a = col_mid_passes_m<N, 0, RE, SIGN, COLS>(a, b, tw, lane);
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
            C w[RE];
#pragma unroll
            for (int r = 1; r < RE; ++r) {
                w[r] = tw[j * r];
                if constexpr (SIGN > 0) w[r].y = -w[r].y;
            }
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                const C* src = in_a ? a[c] : b[c];
#pragma unroll
                for (int r = 0; r < RE; ++r) v[c][q][r] = src[pad8(j + r * NB)];
            }
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
#pragma unroll
                for (int r = 1; r < RE; ++r) v[c][q][r] = cmul(v[c][q][r], w[r]);
                dft<RE, SIGN>(v[c][q]);
            }
        }
    }
}

// ---- twiddles held in registers ------------------------------------------------
// A lane's butterflies, and with them its twiddle factors, are the same in
// every transform of a plan, so a stepper that runs thousands of transforms
// loads them once (ColTw) instead of reading them from LDS in every pass.
template <int N, int P, int NS, typename C, bool END = (P >= ColPlan<N>::NMID)> struct ColTwMid;
template <int N, int P, int NS, typename C> struct ColTwMid<N, P, NS, C, true> {
    __device__ void load(const C*, int) {}
};
template <int N, int P, int NS, typename C> struct ColTwMid<N, P, NS, C, false> {
    static constexpr int R = col_mid_radix(N, ColPlan<N>::MID, P);
    static constexpr int NB = N / R, TS = N / (NS * R), NBL = (NB + kWave - 1) / kWave;
    C w[NBL][R];
    ColTwMid<N, P + 1, NS * R, C> next;
    __device__ void load(const C* tw, int lane) {
#pragma unroll
        for (int b = 0; b < NBL; ++b) {
            const int j = lane + b * kWave;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) w[b][r] = (j < NB && r > 0) ? tw[k * r * TS] : cmk<C>(0, 0);
        }
        next.load(tw, lane);
    }
};
template <int N, typename C> struct ColTw {
    using PL = ColPlan<N>;
    ColTwMid<N, 0, PL::RE, C> mid;
    C last[PL::NBL][PL::RE];
    __device__ void load(const C* tw, int lane) {
        mid.load(tw, lane);
#pragma unroll
        for (int q = 0; q < PL::NBL; ++q) {
            const int j = lane + q * kWave;
#pragma unroll
            for (int r = 0; r < PL::RE; ++r) last[q][r] = (j < PL::NB && r > 0) ? tw[j * r] : cmk<C>(0, 0);
        }
    }
};

template <int SIGN, typename C> __device__ inline C tw_sign(C w) {
    if constexpr (SIGN > 0) w.y = -w.y;
    return w;
}

template <int N, int R, int NS, int SIGN, int COLS, typename C, typename TW>
__device__ inline void col_mid_pass_mr(C* const* in, C* const* out, const TW& t, int lane) {
    constexpr int NB = N / R;
    constexpr int NBL = (NB + kWave - 1) / kWave;
#pragma unroll
    for (int b = 0; b < NBL; ++b) {
        const int j = lane + b * kWave;
        if (j < NB) {
            const int k = j % NS;
            C v[COLS][R];
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) v[c][r] = in[c][pad8(j + r * NB)];
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], tw_sign<SIGN>(t.w[b][r]));
                dft<R, SIGN>(v[c]);
            }
            const int o = (j / NS) * NS * R + k;
#pragma unroll
            for (int c = 0; c < COLS; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) out[c][pad8(o + r * NS)] = v[c][r];
        }
    }
}

template <int N, int P, int NS, int SIGN, int COLS, typename C, typename TW>
__device__ inline bool col_mid_passes_mr(C* const* a, C* const* b, const TW& t, int lane) {
    using PL = ColPlan<N>;
    if constexpr (P >= PL::NMID) {
        return true;  // result in a
    } else {
        constexpr int R = col_mid_radix(N, PL::MID, P);
        col_mid_pass_mr<N, R, NS, SIGN, COLS>(a, b, t, lane);
        wave_lds_sync();
        return !col_mid_passes_mr<N, P + 1, NS * R, SIGN, COLS>(b, a, t.next, lane);
    }
}

// col_fft_m with the twiddles of ColTw (registers).
template <int N, int SIGN, int COLS, typename C>
__device__ inline void col_fft_mr(C (&v)[COLS][ColPlan<N>::NBL][ColPlan<N>::RE], C* const* a, C* const* b,
                                  const ColTw<N, C>& t, int lane) {
    using PL = ColPlan<N>;
    constexpr int RE = PL::RE, NB = PL::NB;
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                dft<RE, SIGN>(v[c][q]);
#pragma unroll
                for (int r = 0; r < RE; ++r) a[c][pad8(j * RE + r)] = v[c][q][r];
            }
        }
    }
    wave_lds_sync();
    const bool in_a = col_mid_passes_mr<N, 0, RE, SIGN, COLS>(a, b, t.mid, lane);
#pragma unroll
    for (int q = 0; q < PL::NBL; ++q) {
        const int j = lane + q * kWave;
        if (j < NB) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                const C* src = in_a ? a[c] : b[c];
#pragma unroll
                for (int r = 0; r < RE; ++r) v[c][q][r] = src[pad8(j + r * NB)];
            }
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
#pragma unroll
                for (int r = 1; r < RE; ++r) v[c][q][r] = cmul(v[c][q][r], tw_sign<SIGN>(t.last[q][r]));
                dft<RE, SIGN>(v[c][q]);
            }
        }
    }
}

// Buffer that col_fft's last pass reads from (the first pass writes `a`).
template <int N> constexpr bool col_result_in_a() { return (ColPlan<N>::NMID % 2) == 0; }

}  // namespace tsk
