// Linearized 2D Navier-Stokes operator (vorticity form) about a parallel base
// flow, pseudo-spectral with the 2/3 rule, integrating-factor RK4 time stepper.
//
// Equation (Sec. 3, eq. "linearized Navier-Stokes equations", curl taken):
//     d omega/dt = -(U d_x omega + v dOmega/dy) + Re^-1 lap omega,
// for a base flow (U(y), 0) with base-vorticity gradient dOmega/dy = -U''(y);
// u = d psi/dy, v = -d psi/dx, -lap psi = omega.  The matvec of the
// exponential propagator M = exp(A T) (Sec. 3.2) is T/dt steps of Lawson's
// integrating-factor RK4 with E(t) = exp(-K^2 t / Re).
//
// MI355X design.  With a base flow that depends on y only, the grid products
// U(y) f(x, y) never mix x-wavenumbers: the forward and inverse x-transforms
// around the product cancel exactly on the kept modes, so each dealiased kx
// column evolves on its own.  One 64-lane workgroup owns one column for the
// whole matvec (all T/dt steps and 4 stages): the column's spectral state, RK
// accumulator and stage input live in registers in the layout of the first and
// last passes of the y-transforms (colfft.hpp), so the spectral bookkeeping and
// the product with the base profile never go through LDS; only the interior
// transform passes do.  HBM is touched only to read the input column once and
// to write the output column once.  No grid-wide
// synchronisation is needed, so a matvec is a single launch of M+1 workgroups.
// When dOmega/dy = c U (true for the Kolmogorov base sin(n y), c = n^2) the two
// inverse transforms are merged in spectral space by linearity,
// d_x omega - c d_x psi <-> i kx (1 - c/K^2) omega_hat.
//
// State layout ("packed spectral", see tsk.h): kx = 0 column jy = 1..M, then
// kx = 1..M columns jy = -M..M, each (re, im) of sqrt(2) rfft2(omega)/N^2.
#include <cmath>
#include <vector>

#include <algorithm>
#include <cstring>
#include <map>
#include <limits>
#include <mutex>
#include <tuple>

#include "colbloch.hpp"
#include "colcouple.hpp"
#include "colcouple_adj.hpp"
#include "colstep.hpp"
#include "kolmo2d.hpp"
#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

// ---- physical <-> packed spectral ------------------------------------------------------
// Z is the N x (M+1) complex intermediate, row-major [y][kx].
template <typename real, int N>
__global__ __launch_bounds__(kWave) void k_rows_fwd(const real* __restrict__ phys, cplx<real>* __restrict__ Z,
                                                    const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    constexpr int M = Geo<N>::M;
    __shared__ C sA[N], sB[N], sT[N];
    const int lane = threadIdx.x, y = blockIdx.x;
    for (int t = lane; t < N; t += kWave) {
        sT[t] = twg[t];
        sA[t] = cmk<C>(phys[size_t(y) * N + t], real(0));
    }
    __syncthreads();
    C* X = fft_lds<N, -1, kWave>(sA, sB, sT, lane);
    for (int kx = lane; kx <= M; kx += kWave) Z[size_t(y) * (M + 1) + kx] = X[kx];
}

template <typename real, int N>
__global__ __launch_bounds__(kWave) void k_cols_fwd(const cplx<real>* __restrict__ Z, real* __restrict__ state,
                                                    const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    using G = Geo<N>;
    constexpr int M = G::M, NM = G::NM;
    __shared__ C sA[N], sB[N], sT[N];
    const int lane = threadIdx.x, kx = blockIdx.x;
    for (int t = lane; t < N; t += kWave) {
        sT[t] = twg[t];
        sA[t] = Z[size_t(t) * (M + 1) + kx];
    }
    __syncthreads();
    C* X = fft_lds<N, -1, kWave>(sA, sB, sT, lane);
    const real sc = real(1.4142135623730950488 / (double(N) * N));
    real* out = state + G::seg(kx);
    if (kx == 0) {
        for (int jy = 1 + lane; jy <= M; jy += kWave) {
            out[2 * (jy - 1)] = X[jy].x * sc;
            out[2 * (jy - 1) + 1] = X[jy].y * sc;
        }
    } else {
        for (int q = lane; q < NM; q += kWave) {
            int jy = q - M, pp = jy < 0 ? jy + N : jy;
            out[2 * q] = X[pp].x * sc;
            out[2 * q + 1] = X[pp].y * sc;
        }
    }
}

template <typename real, int N>
__global__ __launch_bounds__(kWave) void k_cols_inv(const real* __restrict__ state, cplx<real>* __restrict__ Z,
                                                    const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    using G = Geo<N>;
    constexpr int M = G::M, NM = G::NM;
    __shared__ C sA[N], sB[N], sT[N];
    const int lane = threadIdx.x, kx = blockIdx.x;
    for (int t = lane; t < N; t += kWave) {
        sT[t] = twg[t];
        sA[t] = cmk<C>(real(0), real(0));
    }
    __syncthreads();
    const real sc = real(0.70710678118654752440);
    const real* in = state + G::seg(kx);
    if (kx == 0) {
        for (int jy = 1 + lane; jy <= M; jy += kWave) {
            C c = cmk<C>(in[2 * (jy - 1)] * sc, in[2 * (jy - 1) + 1] * sc);
            sA[jy] = c;
            sA[N - jy] = cconj(c);
        }
    } else {
        for (int q = lane; q < NM; q += kWave) {
            int jy = q - M, pp = jy < 0 ? jy + N : jy;
            sA[pp] = cmk<C>(in[2 * q] * sc, in[2 * q + 1] * sc);
        }
    }
    __syncthreads();
    C* X = fft_lds<N, +1, kWave>(sA, sB, sT, lane);
    for (int y = lane; y < N; y += kWave) Z[size_t(y) * (M + 1) + kx] = X[y];
}

template <typename real, int N>
__global__ __launch_bounds__(kWave) void k_rows_inv(const cplx<real>* __restrict__ Z, real* __restrict__ phys,
                                                    const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    constexpr int M = Geo<N>::M;
    __shared__ C sA[N], sB[N], sT[N];
    const int lane = threadIdx.x, y = blockIdx.x;
    for (int t = lane; t < N; t += kWave) {
        sT[t] = twg[t];
        sA[t] = cmk<C>(real(0), real(0));
    }
    __syncthreads();
    for (int kx = lane; kx <= M; kx += kWave) {
        C c = Z[size_t(y) * (M + 1) + kx];
        sA[kx] = c;
        if (kx > 0) sA[N - kx] = cconj(c);
    }
    __syncthreads();
    C* X = fft_lds<N, +1, kWave>(sA, sB, sT, lane);
    for (int x = lane; x < N; x += kWave) phys[size_t(y) * N + x] = X[x].x;
}

// ---- dispatch ------------------------------------------------------------------------------
// Columns per wavefront of the stepper: 1, or 2 for N <= kMaxColsPairN (beyond,
// two columns' registers do not fit).  Chosen per (N, precision, base kind,
// launch size) by timing both variants once per process (column_choice); the
// two variants perform the same arithmetic per column, so the choice changes
// only the speed.
constexpr int kMaxColsPairN = 256;
inline int max_cols(int N) { return N <= kMaxColsPairN ? 2 : 1; }

// Task list of one instance: kx = 0 alone, then groups of `cols` columns.
std::vector<ColTask> column_tasks(int inst, int M, int cols) {
    std::vector<ColTask> t;
    t.push_back(ColTask{inst, 0, 1});
    for (int kx = 1; kx <= M; kx += cols) t.push_back(ColTask{inst, kx, std::min(cols, M - kx + 1)});
    return t;
}

struct TuneKey {
    int N, fp32, prop, bucket;
    bool operator<(const TuneKey& o) const {
        return std::tie(N, fp32, prop, bucket) < std::tie(o.N, o.fp32, o.prop, o.bucket);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

// Times launch(1) and launch(2) (each once to warm up, once measured) on stream
// s and caches the faster; launch(c) must be a complete, repeatable matvec.
template <typename F>
tsk_status column_choice(const TuneKey& key, hipStream_t s, F&& launch, int* out) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *out = it->second;
            return TSK_OK;
        }
    }
    if (max_cols(key.N) == 1) {
        *out = 1;
    } else {
        hipEvent_t e0, e1;
        TSK_HIP(hipEventCreate(&e0));
        TSK_HIP(hipEventCreate(&e1));
        float best = 0.0f;
        int bc = 1;
        for (int c = 1; c <= 2; ++c) {
            launch(c);
            TSK_HIP(hipEventRecord(e0, s));
            launch(c);
            TSK_HIP(hipEventRecord(e1, s));
            TSK_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            TSK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (c == 1 || ms < best) {
                best = ms;
                bc = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        TSK_HIP(hipGetLastError());
        *out = bc;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = *out;
    return TSK_OK;
}

int size_bucket(int columns) {
    int b = 0;
    while ((1 << b) < columns) ++b;
    return b;
}

struct KolmoLaunch {
    const void* x;
    void* y;
    const void* tw;
    void* Z;
    hipStream_t s;
};

template <typename real, int N> struct KK {
    using C = cplx<real>;
    template <int COLS>
    static void colstep_c(const ColInst<real>& one, const ColInst<real>* insts, const ColTask* tasks, int ntasks,
                          bool prop, const void* tw, int jstep, hipStream_t s) {
        if (prop)
            hipLaunchKernelGGL((k_colstep<real, N, true, COLS>), dim3(ntasks), dim3(kWave), 0, s, one, insts, tasks,
                               static_cast<const C*>(tw), jstep);
        else
            hipLaunchKernelGGL((k_colstep<real, N, false, COLS>), dim3(ntasks), dim3(kWave), 0, s, one, insts, tasks,
                               static_cast<const C*>(tw), jstep);
    }
    static void colstep_adj(const ColInst<real>& one, const ColTask* tasks, int ntasks, bool prop, const void* tw,
                            hipStream_t s) {
        if (prop)
            hipLaunchKernelGGL((k_colstep_adj<real, N, true>), dim3(ntasks), dim3(kWave), 0, s, one, tasks,
                               static_cast<const C*>(tw));
        else
            hipLaunchKernelGGL((k_colstep_adj<real, N, false>), dim3(ntasks), dim3(kWave), 0, s, one, tasks,
                               static_cast<const C*>(tw));
    }
    static void colstep(const ColInst<real>& one, const ColInst<real>* insts, const ColTask* tasks, int ntasks,
                        bool prop, int cols, const void* tw, int jstep, hipStream_t s) {
        if constexpr (N <= kMaxColsPairN) {
            if (cols == 2) return colstep_c<2>(one, insts, tasks, ntasks, prop, tw, jstep, s);
        }
        colstep_c<1>(one, insts, tasks, ntasks, prop, tw, jstep, s);
    }
    static void fwd(const KolmoLaunch& a) {
        constexpr int M = Geo<N>::M;
        hipLaunchKernelGGL((k_rows_fwd<real, N>), dim3(N), dim3(kWave), 0, a.s, static_cast<const real*>(a.x),
                           static_cast<C*>(a.Z), static_cast<const C*>(a.tw));
        hipLaunchKernelGGL((k_cols_fwd<real, N>), dim3(M + 1), dim3(kWave), 0, a.s,
                           static_cast<const C*>(a.Z), static_cast<real*>(a.y), static_cast<const C*>(a.tw));
    }
    static void inv(const KolmoLaunch& a) {
        constexpr int M = Geo<N>::M;
        hipLaunchKernelGGL((k_cols_inv<real, N>), dim3(M + 1), dim3(kWave), 0, a.s, static_cast<const real*>(a.x),
                           static_cast<C*>(a.Z), static_cast<const C*>(a.tw));
        hipLaunchKernelGGL((k_rows_inv<real, N>), dim3(N), dim3(kWave), 0, a.s, static_cast<const C*>(a.Z),
                           static_cast<real*>(a.y), static_cast<const C*>(a.tw));
    }
};

#define TSK_KOLMO_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

bool kolmo_size_ok(int N) {
    switch (N) {
#define X(n) case n:
        TSK_KOLMO_SIZES(X)
#undef X
        return true;
        default: return false;
    }
}

template <typename real>
void dispatch_colstep(int N, const ColInst<real>& one, const ColInst<real>* insts, const ColTask* tasks, int ntasks,
                      bool prop, int cols, const void* tw, int jstep, hipStream_t s) {
    switch (N) {
#define X(n) case n: KK<real, n>::colstep(one, insts, tasks, ntasks, prop, cols, tw, jstep, s); break;
        TSK_KOLMO_SIZES(X)
#undef X
    }
}
template <typename real>
void dispatch_colstep_adj(int N, const ColInst<real>& one, const ColTask* tasks, int ntasks, bool prop, const void* tw,
                          hipStream_t s) {
    switch (N) {
#define X(n) case n: KK<real, n>::colstep_adj(one, tasks, ntasks, prop, tw, s); break;
        TSK_KOLMO_SIZES(X)
#undef X
    }
}
template <typename real> void dispatch_fwd(int N, const KolmoLaunch& a) {
    switch (N) {
#define X(n) case n: KK<real, n>::fwd(a); break;
        TSK_KOLMO_SIZES(X)
#undef X
    }
}
template <typename real> void dispatch_inv(int N, const KolmoLaunch& a) {
    switch (N) {
#define X(n) case n: KK<real, n>::inv(a); break;
        TSK_KOLMO_SIZES(X)
#undef X
    }
}

// f = (K^2/Re) lam + ex over the packed entries (ex may be null): the forcing
// -Re^-1 lap omega_lam that holds the laminar flow steady, plus an extra field.
template <typename real>
__global__ void k_forcing(const real* __restrict__ lam, const real* __restrict__ ex, real* __restrict__ f, int M,
                          double alpha, double Re) {
    const int NM = 2 * M + 1;
    const int ne = M + M * NM;  // complex entries
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
        int kx, jy;
        if (e < M) {
            kx = 0;
            jy = e + 1;
        } else {
            kx = 1 + (e - M) / NM;
            jy = (e - M) % NM - M;
        }
        const double kxv = alpha * kx;
        const double s = (kxv * kxv + double(jy) * jy) / Re;
        for (int c = 0; c < 2; ++c) {
            double v = s * double(lam[2 * e + c]);
            if (ex) v += double(ex[2 * e + c]);
            f[2 * e + c] = real(v);
        }
    }
}

// Bloch-sector stepper launch for N = 128, 256, 512: `n` instances (grid y),
// insts[ids[.]] of a batch at Arnoldi step jstep, or `one` (insts null, n = 1).
template <typename real>
void launch_bloch_stepper(int N, const ColInst<real>& one, const ColInst<real>* insts, const int* ids, int n,
                          int jstep, const cplx<real>* tw, hipStream_t s) {
    const int M = (N - 1) / 3;
    if (N == 128)
        hipLaunchKernelGGL((k_colstep_bloch_split<real>), dim3(bloch_blocks(M), n), dim3(kWave), 0, s, one, insts,
                           ids, jstep, tw);
    else if (N == 256)
        hipLaunchKernelGGL((k_colstep_bloch<real, 64>), dim3(bloch_blocks(M), n), dim3(kWave), 0, s, one, insts,
                           ids, jstep, tw);
    else
        hipLaunchKernelGGL((k_colstep_bloch<real, 128>), dim3(bloch_blocks(M), n), dim3(kWave), 0, s, one,
                           insts, ids, jstep, tw);
}

// Spectral-coupling stepper launch (colcouple.hpp): `n` instances (grid y),
// insts[ids[.]] of a batch at Arnoldi step jstep, or `one` (insts null, n = 1);
// blocks = couple_blocks of the largest instance, S positions per lane.
template <typename real, int S>
void launch_couple_shape(const ColInst<real>& one, const ColInst<real>* insts, const int* ids, int n, int jstep,
                         int blocks, int wpw, hipStream_t s) {
    const dim3 grid((blocks + wpw - 1) / wpw, n);
    if (wpw == 1)
        hipLaunchKernelGGL((k_colstep_couple<real, S, 1>), grid, dim3(kWave), 0, s, one, insts, ids, jstep);
    else if (wpw == 2)
        hipLaunchKernelGGL((k_colstep_couple<real, S, 2>), grid, dim3(2 * kWave), 0, s, one, insts, ids, jstep);
    else
        hipLaunchKernelGGL((k_colstep_couple<real, S, 4>), grid, dim3(4 * kWave), 0, s, one, insts, ids, jstep);
}
template <typename real>
void launch_couple_stepper(const ColInst<real>& one, const ColInst<real>* insts, const int* ids, int n, int jstep,
                           int blocks, int S, int wpw, hipStream_t s) {
    if (S == 1)
        launch_couple_shape<real, 1>(one, insts, ids, n, jstep, blocks, wpw, s);
    else
        launch_couple_shape<real, 2>(one, insts, ids, n, jstep, blocks, wpw, s);
}

// Transposed coupling stepper (colcouple_adj.hpp), one instance.
template <typename real, int S>
void launch_couple_adj_shape(const ColInst<real>& one, int blocks, int wpw, hipStream_t s) {
    const dim3 grid((blocks + wpw - 1) / wpw);
    if (wpw == 1)
        hipLaunchKernelGGL((k_colstep_couple_adj<real, S, 1>), grid, dim3(kWave), 0, s, one);
    else if (wpw == 2)
        hipLaunchKernelGGL((k_colstep_couple_adj<real, S, 2>), grid, dim3(2 * kWave), 0, s, one);
    else
        hipLaunchKernelGGL((k_colstep_couple_adj<real, S, 4>), grid, dim3(4 * kWave), 0, s, one);
}
template <typename real>
void launch_couple_adj(const ColInst<real>& one, int blocks, int S, int wpw, hipStream_t s) {
    if (S == 1)
        launch_couple_adj_shape<real, 1>(one, blocks, wpw, s);
    else
        launch_couple_adj_shape<real, 2>(one, blocks, wpw, s);
}

// Launch shape of the coupling stepper (wavefronts per workgroup: 1, 2 or 4),
// timed once per (precision, positions per lane, launch size) and process on
// the first real launch, like the column variants; the shapes compute the same
// bits, so the choice never changes results.
struct CoupleKey {
    bool fp32;
    int S, size;
    int prefer;  // the preferred shape of the caller (0: none); single-operator and batch launches keep apart
    bool operator<(const CoupleKey& o) const {
        return std::tie(fp32, S, size, prefer) < std::tie(o.fp32, o.S, o.size, o.prefer);
    }
};
std::mutex g_couple_mu;
std::map<CoupleKey, int> g_couple;

int wave_bucket(int waves) {
    int b = 1;
    while (b < waves) b *= 2;
    return b;
}

// prefer (single-operator launches): the shape kept when its isolated time is
// within 10% of the fastest.  Isolated launches of one operator come out nearly
// even, but inside an Arnoldi run, beside its Gram-Schmidt kernels and Ritz
// analyses, interleaved runs ranked them clearly: FP32 256^2 27.3 us per
// matvec with 4 wavefronts per workgroup, 29.9 with 2, 31.0 with 1 (whole
// solve 7.9 against 8.2 ms); FP64 128^2 and 256^2 fastest with 1.
template <typename F>
tsk_status couple_choice(const CoupleKey& key, hipStream_t s, F&& launch, int* out, int prefer = 0) {
    {
        std::lock_guard<std::mutex> lk(g_couple_mu);
        auto it = g_couple.find(key);
        if (it != g_couple.end()) {
            *out = it->second;
            return TSK_OK;
        }
    }
    hipEvent_t e0, e1;
    TSK_HIP(hipEventCreate(&e0));
    TSK_HIP(hipEventCreate(&e1));
    // one untimed launch per shape, then three rounds over the shapes with one
    // timed launch each; the shortest time of each shape decides (one launch
    // per shape varied by more than the shapes differ)
    constexpr int kShapes[3] = {1, 2, 4};
    float tmin[3] = {0.0f, 0.0f, 0.0f};
    for (int w : kShapes) launch(w);
    for (int round = 0; round < 3; ++round)
        for (int q = 0; q < 3; ++q) {
            TSK_HIP(hipEventRecord(e0, s));
            launch(kShapes[q]);
            TSK_HIP(hipEventRecord(e1, s));
            TSK_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            TSK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (round == 0 || ms < tmin[q]) tmin[q] = ms;
        }
    int bw = kShapes[0];
    float best = tmin[0];
    for (int q = 1; q < 3; ++q)
        if (tmin[q] < best) {
            best = tmin[q];
            bw = kShapes[q];
        }
    for (int q = 0; q < 3; ++q)
        if (kShapes[q] == prefer && tmin[q] <= 1.10f * best) bw = prefer;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TSK_HIP(hipGetLastError());
    *out = bw;
    std::lock_guard<std::mutex> lk(g_couple_mu);
    g_couple[key] = bw;
    return TSK_OK;
}

// Positions per lane of the coupling stepper for cutoff M and harmonic nh: the
// longest chain has ceil((2M + 1) / nh) modes.
inline int couple_slots(int M, int nh) { return ((2 * M + 1 + nh - 1) / nh + kWave - 1) / kWave; }

struct KolmoOp final : Operator {
    int N = 0, M = 0;
    tsk_precision prec = TSK_FP64;
    double alpha = 0.0, Re = 0.0, dt = 0.0;
    int nsteps = 0;
    bool prop = false;
    double cprop = 0.0;
    bool bloch = false;  // N = 128, 256, 512 and a quarter-period one-harmonic profile: Bloch-sector stepper
    // one-harmonic profile U = amp sin(nh (y - y0)): spectral-coupling stepper (colcouple.hpp)
    bool couple = false;
    int nh = 0;
    double amp = 0.0, y0 = 0.0;
    DevBuf tw, negU, dOdy, Z;
    DevBuf tasks[3];   // single-instance task lists for 1 and 2 columns per wavefront
    int ntasks[3] = {0, 0, 0};
    int force_cols = 0;  // 0: automatic choice; 1, 2: column stepper; 3: Bloch-sector stepper
    int force_wpw = 0;   // coupling stepper's wavefronts per workgroup: 0 tuned, else 1, 2 or 4
    int tuned_wpw = 0;   // the tuned (or forced) shape of the last launch
    Gen2D* gen = nullptr;  // general two-dimensional base flow (kolmo2d.hip), else parallel
    // nonlinear forced equation (fixed-point solvers): pipeline workspace, packed
    // forcing and laminar state, drift, and the inputs the forcing is made from
    Gen2D* nlw = nullptr;
    DevBuf fvec, lam, physbuf;
    double U0 = 0.0;
    int nforce = 0;
    std::vector<double> extra;  // extra forcing field (physical, N*N), empty if none
    bool nl_set = false;
    ~KolmoOp() override {
        gen2d_free(gen);
        gen2d_free(nlw);
    }

    const char* name() const override { return "kolmo2d"; }
    int64_t physical_reals() const override { return int64_t(N) * N; }
    size_t rb() const { return prec == TSK_FP32 ? 4 : 8; }

    tsk_status upload_real(DevBuf& buf, const std::vector<double>& v) {
        TSK_TRY(buf.ensure(v.size() * rb()));
        if (prec == TSK_FP32) {
            std::vector<float> f(v.begin(), v.end());
            TSK_HIP(hipMemcpy(buf.ptr, f.data(), f.size() * 4, hipMemcpyHostToDevice));
        } else {
            TSK_HIP(hipMemcpy(buf.ptr, v.data(), v.size() * 8, hipMemcpyHostToDevice));
        }
        return TSK_OK;
    }

    tsk_status init() {
        std::vector<double> t(2 * size_t(N));
        for (int i = 0; i < N; ++i) {
            // exp(-2 pi i t / N), evaluated in FP64 on the host
            const double pi = 3.14159265358979323846264338327950288;
            double ang = 2.0 * pi * double(i) / N;
            t[2 * i] = std::cos(ang);
            t[2 * i + 1] = -std::sin(ang);
        }
        TSK_TRY(upload_real(tw, t));
        TSK_TRY(Z.ensure(size_t(N) * (M + 1) * 2 * rb()));
        for (int c = 1; c <= max_cols(N); ++c) {
            const std::vector<ColTask> tk = column_tasks(0, M, c);
            TSK_TRY(tasks[c].ensure(tk.size() * sizeof(ColTask)));
            TSK_HIP(hipMemcpy(tasks[c].ptr, tk.data(), tk.size() * sizeof(ColTask), hipMemcpyHostToDevice));
            ntasks[c] = int(tk.size());
        }
        return TSK_OK;
    }

    KolmoLaunch args(const void* x, void* y) const {
        KolmoLaunch a{x, y, tw.ptr, Z.ptr, stream};
        return a;
    }

    template <typename real> ColInst<real> inst(const void* xbase, int64_t xstride, void* y, const int* act) const {
        ColInst<real> c;
        c.xbase = static_cast<const real*>(xbase);
        c.xstride = xstride;
        c.y = static_cast<real*>(y);
        c.negU = negU.as<real>();
        c.dOdy = dOdy.as<real>();
        c.alpha = alpha;
        c.Re = Re;
        c.dt = dt;
        c.cprop = cprop;
        c.nsteps = nsteps;
        c.active = act;
        c.M = M;
        c.nh = nh;
        c.amp = amp;
        c.y0 = y0;
        c.jmax = std::numeric_limits<int>::max();
        return c;
    }
    bool use_couple() const { return !gen && couple && force_cols == 0; }
    bool use_bloch() const { return !gen && bloch && (force_cols == 3 || (force_cols == 0 && !couple)); }

    template <typename real> void launch_bloch(const void* x, void* y) const {
        launch_bloch_stepper<real>(N, inst<real>(x, 0, y, nullptr), nullptr, nullptr, 1, 0, tw.as<cplx<real>>(),
                                   stream);
    }
    tsk_status apply(const void* x, void* y) override {
        if (!ready()) return fail(TSK_ESTATE, "Navier-Stokes parameters or base flow not set");
        if (x == y) return fail(TSK_EINVAL, "apply: input and output must not alias");
        if (gen) return gen2d_apply(gen, alpha, Re, dt, nsteps, x, y, tw.ptr, stream);
        if (use_couple()) {
            const int S = couple_slots(M, nh), blocks = couple_blocks(M, nh);
            auto launch = [&](int w) {
                if (prec == TSK_FP32)
                    launch_couple_stepper<float>(inst<float>(x, 0, y, nullptr), nullptr, nullptr, 1, 0, blocks, S, w,
                                                 stream);
                else
                    launch_couple_stepper<double>(inst<double>(x, 0, y, nullptr), nullptr, nullptr, 1, 0, blocks, S, w,
                                                  stream);
            };
            int w = force_wpw;
            if (w == 0) {
                const int prefer = prec == TSK_FP32 ? 4 : 1;
                TSK_TRY(couple_choice(CoupleKey{prec == TSK_FP32, S, wave_bucket(blocks), prefer}, stream, launch, &w,
                                      prefer));
            }
            tuned_wpw = w;
            launch(w);
            TSK_HIP(hipGetLastError());
            return TSK_OK;
        }
        if (use_bloch()) {
            if (prec == TSK_FP32)
                launch_bloch<float>(x, y);
            else
                launch_bloch<double>(x, y);
            TSK_HIP(hipGetLastError());
            return TSK_OK;
        }
        auto launch = [&](int c) {
            if (prec == TSK_FP32)
                dispatch_colstep<float>(N, inst<float>(x, 0, y, nullptr), nullptr, tasks[c].as<ColTask>(), ntasks[c],
                                        prop, c, tw.ptr, 0, stream);
            else
                dispatch_colstep<double>(N, inst<double>(x, 0, y, nullptr), nullptr, tasks[c].as<ColTask>(),
                                         ntasks[c], prop, c, tw.ptr, 0, stream);
        };
        int cols = std::min(force_cols, max_cols(N));
        if (cols == 0)
            TSK_TRY(column_choice(TuneKey{N, prec == TSK_FP32, prop, size_bucket(M + 1)}, stream, launch, &cols));
        launch(cols);
        TSK_HIP(hipGetLastError());
        return TSK_OK;
    }
    bool has_adjoint() const override { return true; }
    // Transposed propagator: for a one-harmonic base the transposed coupling
    // stepper (k_colstep_couple_adj, in the launch shape the forward stepper
    // kept, else one wavefront per workgroup); other parallel bases the
    // transposed column stepper (k_colstep_adj, task list of 1-column tasks);
    // a general 2-D base the transposed pipeline of kolmo2d.hip.
    tsk_status apply_adjoint(const void* x, void* y) override {
        if (!ready()) return fail(TSK_ESTATE, "Navier-Stokes parameters or base flow not set");
        if (x == y) return fail(TSK_EINVAL, "apply_adjoint: input and output must not alias");
        if (gen) return gen2d_apply_adjoint(gen, alpha, Re, dt, nsteps, x, y, tw.ptr, stream);
        if (use_couple()) {
            const int S = couple_slots(M, nh), blocks = couple_blocks(M, nh);
            const int w = force_wpw ? force_wpw : (tuned_wpw ? tuned_wpw : 1);
            if (prec == TSK_FP32)
                launch_couple_adj<float>(inst<float>(x, 0, y, nullptr), blocks, S, w, stream);
            else
                launch_couple_adj<double>(inst<double>(x, 0, y, nullptr), blocks, S, w, stream);
            TSK_HIP(hipGetLastError());
            return TSK_OK;
        }
        if (prec == TSK_FP32)
            dispatch_colstep_adj<float>(N, inst<float>(x, 0, y, nullptr), tasks[1].as<ColTask>(), ntasks[1], prop,
                                        tw.ptr, stream);
        else
            dispatch_colstep_adj<double>(N, inst<double>(x, 0, y, nullptr), tasks[1].as<ColTask>(), ntasks[1], prop,
                                         tw.ptr, stream);
        TSK_HIP(hipGetLastError());
        return TSK_OK;
    }
    // physical N*N field (host FP64) -> packed state (device) through physbuf
    tsk_status pack_host_field(const std::vector<double>& f, void* state) {
        TSK_TRY(upload_real(physbuf, f));
        return from_physical(physbuf.ptr, state);
    }
    // forcing from nforce, Re and the extra field (needs Re)
    tsk_status make_forcing() {
        const size_t sb = state_bytes();
        std::vector<double> w(size_t(N) * N);
        const double pi = 3.14159265358979323846264338327950288;
        for (int l = 0; l < N; ++l) {
            const double y = 2.0 * pi * l / N;
            for (int i = 0; i < N; ++i) w[size_t(l) * N + i] = -nforce * std::cos(nforce * y);
        }
        TSK_TRY(lam.ensure(sb));
        TSK_TRY(fvec.ensure(sb));
        TSK_TRY(pack_host_field(w, lam.ptr));
        DevBuf exs;
        if (!extra.empty()) {
            TSK_TRY(exs.ensure(sb));
            TSK_TRY(pack_host_field(extra, exs.ptr));
        }
        if (prec == TSK_FP32)
            hipLaunchKernelGGL(k_forcing<float>, dim3(64), dim3(256), 0, stream, lam.as<float>(),
                               extra.empty() ? nullptr : exs.as<float>(), fvec.as<float>(), M, alpha, Re);
        else
            hipLaunchKernelGGL(k_forcing<double>, dim3(64), dim3(256), 0, stream, lam.as<double>(),
                               extra.empty() ? nullptr : exs.as<double>(), fvec.as<double>(), M, alpha, Re);
        TSK_HIP(hipGetLastError());
        TSK_HIP(hipStreamSynchronize(stream));  // exs is freed on return
        return TSK_OK;
    }
    tsk_status nonlinear_step(const void* x, void* y, int steps) {
        if (!nl_set) return fail(TSK_ESTATE, "nonlinear equation not set (tsk_set_nonlinear)");
        return gen2d_nonlinear(nlw, alpha, Re, dt, steps > 0 ? steps : nsteps, U0, fvec.ptr, x, y, tw.ptr, stream);
    }
    // the general base flow becomes the state x (its grid fields)
    tsk_status base_from_state(const void* x) {
        Gen2D* g = nullptr;
        TSK_TRY(gen2d_create(N, prec == TSK_FP32, nullptr, nullptr, nullptr, nullptr, &g));
        const tsk_status st = gen2d_fields(g, alpha, nl_set ? U0 : 0.0, x, tw.ptr, stream);
        if (st != TSK_OK) {
            gen2d_free(g);
            return st;
        }
        gen2d_free(gen);
        gen = g;
        base_set = true;
        return TSK_OK;
    }
    tsk_status from_physical(const void* phys, void* state) override {
        KolmoLaunch a = args(phys, state);
        if (prec == TSK_FP32) dispatch_fwd<float>(N, a);
        else dispatch_fwd<double>(N, a);
        TSK_HIP(hipGetLastError());
        return TSK_OK;
    }
    tsk_status to_physical(const void* state, void* phys) override {
        KolmoLaunch a = args(state, phys);
        if (prec == TSK_FP32) dispatch_inv<float>(N, a);
        else dispatch_inv<double>(N, a);
        TSK_HIP(hipGetLastError());
        return TSK_OK;
    }
};

}  // namespace

tsk_status make_kolmo(int N, tsk_precision prec, hipStream_t s, std::unique_ptr<Operator>* out) {
    if (!kolmo_size_ok(N))
        return fail(TSK_EINVAL, "grid size N must be one of 16, 32, 48, 64, 96, 128, 192, 256, 384, 512");
    if (prec != TSK_FP64 && prec != TSK_FP32) return fail(TSK_EINVAL, "unknown precision");
    auto op = std::make_unique<KolmoOp>();
    op->N = N;
    op->M = (N - 1) / 3;
    op->prec = prec;
    op->stream = s;
    op->n = 4ll * op->M * (op->M + 1);
    op->kind = prec == TSK_FP32 ? StateKind::Real32 : StateKind::Real64;
    TSK_TRY(op->init());
    *out = std::move(op);
    return TSK_OK;
}

tsk_status kolmo_set_params(Operator* op, double Re, double alpha, double dt, double T) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!(Re > 0.0) || !(alpha > 0.0) || !(dt > 0.0) || !(T > 0.0) || !std::isfinite(Re) || !std::isfinite(alpha) ||
        !std::isfinite(dt) || !std::isfinite(T))
        return fail(TSK_EINVAL, "Re, alpha, dt and T must be positive and finite");
    double ns = T / dt;
    int nsi = int(std::lround(ns));
    if (nsi < 1 || std::fabs(ns - nsi) > 1e-9 * std::max(1.0, ns))
        return fail(TSK_EINVAL, "T must be an integer multiple of dt");
    k->Re = Re;
    k->alpha = alpha;
    k->dt = dt;
    k->nsteps = nsi;
    k->T = T;
    k->params_set = true;
    if (k->nl_set) TSK_TRY(k->make_forcing());
    return TSK_OK;
}

tsk_status kolmo_set_nonlinear(Operator* op, int n_forcing, double U0, const double* extra) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!k->params_set) return fail(TSK_ESTATE, "set Re, alpha, dt and T first");
    if (n_forcing < 1 || n_forcing > k->M) return fail(TSK_EINVAL, "forcing wavenumber must be in [1, (N-1)/3]");
    if (!std::isfinite(U0)) return fail(TSK_EINVAL, "drift must be finite");
    const size_t nn = size_t(k->N) * k->N;
    if (extra)
        for (size_t i = 0; i < nn; ++i)
            if (!std::isfinite(extra[i])) return fail(TSK_ENONFINITE, "non-finite extra forcing");
    if (!k->nlw) TSK_TRY(gen2d_create(k->N, k->prec == TSK_FP32, nullptr, nullptr, nullptr, nullptr, &k->nlw));
    k->nforce = n_forcing;
    k->U0 = U0;
    if (extra)
        k->extra.assign(extra, extra + nn);
    else
        k->extra.clear();
    TSK_TRY(k->make_forcing());
    k->nl_set = true;
    return TSK_OK;
}

tsk_status kolmo_nonlinear_step(Operator* op, const void* x, void* y, int nsteps) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (nsteps < 0) return fail(TSK_EINVAL, "nsteps must be >= 0");
    return k->nonlinear_step(x, y, nsteps);
}

tsk_status kolmo_laminar_state(Operator* op, void* x) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!k->nl_set) return fail(TSK_ESTATE, "nonlinear equation not set (tsk_set_nonlinear)");
    TSK_HIP(hipMemcpyAsync(x, k->lam.ptr, k->state_bytes(), hipMemcpyDeviceToDevice, k->stream));
    return TSK_OK;
}

tsk_status kolmo_base_from_state(Operator* op, const void* x) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!k->params_set) return fail(TSK_ESTATE, "set Re, alpha, dt and T first");
    return k->base_from_state(x);
}

double kolmo_dt(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k ? k->dt : 0.0;
}

int kolmo_nsteps(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k ? k->nsteps : 0;
}

tsk_status kolmo_set_base_parallel(Operator* op, const double* U, const double* dOdy) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!U || !dOdy) return fail(TSK_EINVAL, "null base-flow profile");
    const int N = k->N;
    std::vector<double> nu(N), oy(N);
    double uu = 0.0, uo = 0.0, omax = 0.0;
    for (int i = 0; i < N; ++i) {
        if (!std::isfinite(U[i]) || !std::isfinite(dOdy[i])) return fail(TSK_ENONFINITE, "non-finite base flow");
        nu[i] = -U[i];
        oy[i] = dOdy[i];
        uu += U[i] * U[i];
        uo += U[i] * dOdy[i];
        omax = std::max(omax, std::fabs(dOdy[i]));
    }
    // detect dOmega/dy = c U (one inverse transform per stage instead of two)
    double c = uu > 0.0 ? uo / uu : 0.0;
    double dev = 0.0;
    for (int i = 0; i < N; ++i) dev = std::max(dev, std::fabs(dOdy[i] - c * U[i]));
    k->prop = uu > 0.0 && dev <= 1e-13 * std::max(omax, 1e-300);
    k->cprop = k->prop ? c : 0.0;
    // Bloch sectors (colbloch.hpp): N = 128, 256 or 512, profile of period L = N/4
    // samples whose L-point spectrum has no harmonic beyond the first
    k->bloch = false;
    if (k->prop && (N == 128 || N == 256 || N == 512)) {
        const int L = N / 4;
        double umax = 0.0;
        for (int i = 0; i < N; ++i) umax = std::max(umax, std::fabs(nu[i]));
        bool ok = umax > 0.0;
        for (int i = L; i < N && ok; ++i) ok = std::fabs(nu[i] - nu[i % L]) <= 1e-13 * umax;
        const double pi = 3.14159265358979323846264338327950288;
        for (int h = 2; h <= L / 2 && ok; ++h) {
            double cr = 0.0, ci = 0.0;
            for (int b = 0; b < L; ++b) {
                cr += nu[b] * std::cos(2.0 * pi * h * b / L);
                ci -= nu[b] * std::sin(2.0 * pi * h * b / L);
            }
            ok = std::hypot(cr, ci) <= 1e-12 * L * umax;
        }
        k->bloch = ok;
    }
    // one harmonic (colcouple.hpp): U = amp sin(nh (y - y0)), zero mean, no other
    // harmonic on the N-point grid (to 1e-12 of the amplitude); exact when no term
    // of the product wraps onto a kept mode (nh < N - 2M) and every chain fits two
    // positions per lane
    k->couple = false;
    if (k->prop) {
        const double pi = 3.14159265358979323846264338327950288;
        double umax = 0.0;
        for (int i = 0; i < N; ++i) umax = std::max(umax, std::fabs(U[i]));
        int hsel = 0, nbig = 0;
        double hr = 0.0, hi = 0.0, amax = 0.0;
        std::vector<double> mag(N / 2 + 1);
        for (int h = 0; h <= N / 2; ++h) {
            double cr = 0.0, ci = 0.0;
            for (int l = 0; l < N; ++l) {
                const double a = 2.0 * pi * double(h) * l / N;
                cr += U[l] * std::cos(a);
                ci -= U[l] * std::sin(a);
            }
            mag[h] = std::hypot(cr, ci) / N;  // |U_h|, U(y) = sum_h U_h e^{i h y}
            if (mag[h] > amax) { amax = mag[h]; hsel = h; hr = cr / N; hi = ci / N; }
        }
        for (int h = 0; h <= N / 2; ++h) nbig += mag[h] > 1e-12 * amax ? 1 : 0;
        const int M = k->M;
        if (umax > 0.0 && nbig == 1 && hsel >= 1 && hsel < N / 2 && hsel < N - 2 * M &&
            couple_slots(M, hsel) <= 2) {
            // U = 2 Re(U_h e^{i h y}) = 2|U_h| cos(h y + theta) = amp sin(h (y - y0))
            const double theta = std::atan2(hi, hr);
            k->couple = true;
            k->nh = hsel;
            k->amp = 2.0 * std::hypot(hr, hi);
            k->y0 = -(theta + 0.5 * pi) / hsel;
            if (std::fabs(k->y0) < 1e-15) k->y0 = 0.0;
        }
    }
    TSK_TRY(k->upload_real(k->negU, nu));
    TSK_TRY(k->upload_real(k->dOdy, oy));
    gen2d_free(k->gen);
    k->gen = nullptr;
    k->base_set = true;
    return TSK_OK;
}

tsk_status kolmo_set_base_general(Operator* op, const double* U, const double* V, const double* Ox,
                                  const double* Oy) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (!U || !V || !Ox || !Oy) return fail(TSK_EINVAL, "null base-flow field");
    const size_t nn = size_t(k->N) * k->N;
    for (const double* f : {U, V, Ox, Oy})
        for (size_t i = 0; i < nn; ++i)
            if (!std::isfinite(f[i])) return fail(TSK_ENONFINITE, "non-finite base flow");
    Gen2D* g = nullptr;
    TSK_TRY(gen2d_create(k->N, k->prec == TSK_FP32, U, V, Ox, Oy, &g));
    gen2d_free(k->gen);
    k->gen = g;
    k->base_set = true;
    return TSK_OK;
}

tsk_status kolmo_set_tuning(Operator* op, int cols) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (cols < 0 || cols > 3)
        return fail(TSK_EINVAL, "tuning must be 0 (automatic), 1 or 2 (columns per wavefront) or 3 (Bloch sectors)");
    k->force_cols = cols;
    return TSK_OK;
}

tsk_status kolmo_get_tuning(const Operator* op, int* cols) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (k->use_couple()) {
        *cols = -2;  // the spectral-coupling stepper
        return TSK_OK;
    }
    if (k->use_bloch()) {
        *cols = -1;  // the Bloch-sector stepper
        return TSK_OK;
    }
    int c = std::min(k->force_cols, max_cols(k->N));
    if (c == 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(TuneKey{k->N, k->prec == TSK_FP32, k->prop, size_bucket(k->M + 1)});
        c = it == g_tune.end() ? 0 : it->second;
    }
    *cols = c;
    return TSK_OK;
}

tsk_status kolmo_set_stepper_waves(Operator* op, int w) {
    auto* k = dynamic_cast<KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    if (w != 0 && w != 1 && w != 2 && w != 4)
        return fail(TSK_EINVAL, "wavefronts per workgroup must be 0 (tuned), 1, 2 or 4");
    k->force_wpw = w;
    return TSK_OK;
}

tsk_status kolmo_get_stepper_waves(const Operator* op, int* w) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    if (!k) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
    *w = k->force_wpw ? k->force_wpw : k->tuned_wpw;
    return TSK_OK;
}

bool kolmo_parallel(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k && !k->gen;
}

bool is_kolmo(const Operator* op) { return dynamic_cast<const KolmoOp*>(op) != nullptr; }

bool kolmo_bloch(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k && k->use_bloch();
}

bool kolmo_couple(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k && k->use_couple();
}

int kolmo_cutoff(const Operator* op) {
    const auto* k = dynamic_cast<const KolmoOp*>(op);
    return k ? k->M : -1;
}

// ---- batched matvec -----------------------------------------------------------------------------
// One launch per (N, base kind, stepper) group, all instances of the batch in
// one instance table: the column stepper with a task per (instance, kx column),
// or the Bloch-sector stepper (instances whose single matvec would use it) with
// the group's instance indices on grid y.
struct KolmoBatch {
    bool fp32 = false;
    DevBuf insts;
    std::vector<char> host_insts;  // the instance table as uploaded (restart offsets rewrite it)
    struct Group {
        int N;
        bool prop;
        bool bloch = false;
        bool couple = false;  // spectral-coupling stepper: instances of every N in one launch
        int cblocks = 0, cslots = 1;  // its grid x (largest instance) and positions per lane
        int cwpw = 1;                 // its launch shape (wavefronts per workgroup, tuned)
        DevBuf ids;  // Bloch and coupling groups: instance indices
        int nids = 0;
        const void* tw;
        DevBuf tasks[3];  // task lists for 1 and 2 columns per wavefront
        int ntasks[3] = {0, 0, 0};
        int cols = 1;     // chosen variant
        int force = 0;
        int columns = 0;  // kx columns of all instances
        double work;
    };
    std::vector<std::unique_ptr<Group>> groups;
    // groups after the first run on the process's worker streams 1 and 2
    // (borrowed, not owned; the Arnoldi driver then analyses on stream 0 only),
    // forked from and joined back into the caller's stream
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
    ~KolmoBatch() {
        for (hipEvent_t e : done) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
    }
};

tsk_status kolmo_batch_plan(Operator* const* ops, int count, const KryDesc* Dh, const KryDesc* Dd,
                            KolmoBatchPtr* out) {
    auto b = std::make_unique<KolmoBatch>();
    std::vector<KolmoOp*> ko(count);
    for (int i = 0; i < count; ++i) {
        ko[i] = dynamic_cast<KolmoOp*>(ops[i]);
        if (!ko[i]) return fail(TSK_EINVAL, "batched matvec needs Navier-Stokes operators");
        if (ko[i]->prec != ko[0]->prec) return fail(TSK_EINVAL, "a batch must share one precision");
    }
    b->fp32 = ko[0]->prec == TSK_FP32;
    const size_t isz = b->fp32 ? sizeof(ColInst<float>) : sizeof(ColInst<double>);
    std::vector<char> host(isz * count);
    for (int i = 0; i < count; ++i) {
        const int* act = &Dd[i].active;  // device address of the instance's flag
        if (b->fp32) {
            ColInst<float> c = ko[i]->inst<float>(Dh[i].V, Dh[i].ldv, Dh[i].w, act);
            std::memcpy(host.data() + isz * i, &c, isz);
        } else {
            ColInst<double> c = ko[i]->inst<double>(Dh[i].V, Dh[i].ldv, Dh[i].w, act);
            std::memcpy(host.data() + isz * i, &c, isz);
        }
    }
    TSK_TRY(b->insts.ensure(host.size()));
    TSK_HIP(hipMemcpy(b->insts.ptr, host.data(), host.size(), hipMemcpyHostToDevice));
    b->host_insts = host;
    std::vector<std::vector<int>> gids;
    for (int i = 0; i < count; ++i) {
        const bool kc = kolmo_couple(ko[i]);
        const bool kb = !kc && kolmo_bloch(ko[i]);
        KolmoBatch::Group* g = nullptr;
        for (size_t q = 0; q < b->groups.size() && !g; ++q) {
            KolmoBatch::Group* c = b->groups[q].get();
            if ((kc && c->couple) ||
                (!kc && !c->couple && c->N == ko[i]->N && c->prop == ko[i]->prop && c->bloch == kb)) {
                g = c;
                gids[q].push_back(i);
            }
        }
        if (!g) {
            b->groups.push_back(std::make_unique<KolmoBatch::Group>());
            gids.push_back({i});
            g = b->groups.back().get();
            g->N = ko[i]->N;
            g->prop = ko[i]->prop;
            g->bloch = kb;
            g->couple = kc;
            g->tw = ko[i]->tw.ptr;
            g->force = ko[i]->force_cols;
        }
        g->columns += ko[i]->M + 1;
        if (kc) {
            g->cblocks = std::max(g->cblocks, couple_blocks(ko[i]->M, ko[i]->nh));
            g->cslots = std::max(g->cslots, couple_slots(ko[i]->M, ko[i]->nh));
            if (ko[i]->force_wpw) g->cwpw = ko[i]->force_wpw;
            g->force = g->force ? g->force : ko[i]->force_wpw;
        }
    }
    for (size_t q = 0; q < b->groups.size(); ++q) {
        KolmoBatch::Group* g = b->groups[q].get();
        if (!g->bloch && !g->couple) continue;
        g->nids = int(gids[q].size());
        TSK_TRY(g->ids.ensure(gids[q].size() * sizeof(int)));
        TSK_HIP(hipMemcpy(g->ids.ptr, gids[q].data(), gids[q].size() * sizeof(int), hipMemcpyHostToDevice));
    }
    for (auto& g : b->groups)
        g->work = g->couple ? double(g->columns) * g->cslots * kWave : double(g->columns) * g->N * std::log2(double(g->N));
    std::sort(b->groups.begin(), b->groups.end(),
              [](const std::unique_ptr<KolmoBatch::Group>& x, const std::unique_ptr<KolmoBatch::Group>& y) {
                  return x->work > y->work;
              });
    hipStream_t pool[ArnoldiWork::kAnaStreams];
    if (b->groups.size() > 1) TSK_TRY(analysis_streams(pool));
    for (size_t q = 1; q < b->groups.size(); ++q) {
        hipEvent_t ev;
        b->aux.push_back(pool[1 + (q - 1) % (ArnoldiWork::kAnaStreams - 1)]);
        TSK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->done.push_back(ev);
    }
    if (b->groups.size() > 1) TSK_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    const hipStream_t s = ops[0]->stream;
    for (auto& g : b->groups) {
        if (g->couple) {
            // the launch shape: forced by an instance of the group, else timed on the
            // step-0 inputs (the outputs are overwritten by the first real matvec)
            if (g->force) continue;
            KolmoBatch::Group* gp = g.get();
            KolmoBatch* bp = b.get();
            auto launch = [&](int w) {
                if (bp->fp32)
                    launch_couple_stepper<float>(ColInst<float>{}, bp->insts.as<ColInst<float>>(), gp->ids.as<int>(),
                                                 gp->nids, 0, gp->cblocks, gp->cslots, w, s);
                else
                    launch_couple_stepper<double>(ColInst<double>{}, bp->insts.as<ColInst<double>>(),
                                                  gp->ids.as<int>(), gp->nids, 0, gp->cblocks, gp->cslots, w, s);
            };
            TSK_TRY(couple_choice(CoupleKey{b->fp32, g->cslots, wave_bucket(g->cblocks * g->nids), 0}, s, launch,
                                  &g->cwpw));
            continue;
        }
        if (g->bloch) continue;  // no column tasks, nothing to tune
        for (int c = 1; c <= max_cols(g->N); ++c) {
            std::vector<ColTask> tk;
            for (int i = 0; i < count; ++i)
                if (ko[i]->N == g->N && ko[i]->prop == g->prop) {
                    const std::vector<ColTask> ti = column_tasks(i, ko[i]->M, c);
                    tk.insert(tk.end(), ti.begin(), ti.end());
                }
            TSK_TRY(g->tasks[c].ensure(tk.size() * sizeof(ColTask)));
            TSK_HIP(hipMemcpy(g->tasks[c].ptr, tk.data(), tk.size() * sizeof(ColTask), hipMemcpyHostToDevice));
            g->ntasks[c] = int(tk.size());
        }
        // the variant: forced by the first operator of the group, else timed on the
        // step-0 inputs (the outputs are overwritten by the first real matvec)
        KolmoBatch::Group* gp = g.get();
        KolmoBatch* bp = b.get();
        auto launch = [&](int c) {
            if (bp->fp32)
                dispatch_colstep<float>(gp->N, ColInst<float>{}, bp->insts.as<ColInst<float>>(),
                                        gp->tasks[c].as<ColTask>(), gp->ntasks[c], gp->prop, c, gp->tw, 0, s);
            else
                dispatch_colstep<double>(gp->N, ColInst<double>{}, bp->insts.as<ColInst<double>>(),
                                         gp->tasks[c].as<ColTask>(), gp->ntasks[c], gp->prop, c, gp->tw, 0, s);
        };
        g->cols = std::min(g->force, max_cols(g->N));
        if (g->cols == 0)
            TSK_TRY(column_choice(TuneKey{g->N, b->fp32, g->prop, size_bucket(g->columns)}, s, launch, &g->cols));
    }
    out->reset(b.release());
    return TSK_OK;
}

tsk_status kolmo_batch_matvec(KolmoBatch* b, int j, hipStream_t s) {
    const size_t G = b->groups.size();
    if (G > 1) TSK_HIP(hipEventRecord(b->fork, s));
    for (size_t q = 0; q < G; ++q) {
        auto& g = b->groups[q];
        hipStream_t st = q == 0 ? s : b->aux[q - 1];
        if (q > 0) TSK_HIP(hipStreamWaitEvent(st, b->fork, 0));
        const int c = g->cols;
        if (g->couple) {
            if (b->fp32)
                launch_couple_stepper<float>(ColInst<float>{}, b->insts.as<ColInst<float>>(), g->ids.as<int>(),
                                             g->nids, j, g->cblocks, g->cslots, g->cwpw, st);
            else
                launch_couple_stepper<double>(ColInst<double>{}, b->insts.as<ColInst<double>>(), g->ids.as<int>(),
                                              g->nids, j, g->cblocks, g->cslots, g->cwpw, st);
        } else if (g->bloch) {
            if (b->fp32)
                launch_bloch_stepper<float>(g->N, ColInst<float>{}, b->insts.as<ColInst<float>>(), g->ids.as<int>(),
                                            g->nids, j, static_cast<const cplx<float>*>(g->tw), st);
            else
                launch_bloch_stepper<double>(g->N, ColInst<double>{}, b->insts.as<ColInst<double>>(),
                                             g->ids.as<int>(), g->nids, j, static_cast<const cplx<double>*>(g->tw), st);
        } else if (b->fp32)
            dispatch_colstep<float>(g->N, ColInst<float>{}, b->insts.as<ColInst<float>>(), g->tasks[c].as<ColTask>(),
                                    g->ntasks[c], g->prop, c, g->tw, j, st);
        else
            dispatch_colstep<double>(g->N, ColInst<double>{}, b->insts.as<ColInst<double>>(),
                                     g->tasks[c].as<ColTask>(), g->ntasks[c], g->prop, c, g->tw, j, st);
        TSK_HIP(hipGetLastError());
        if (q > 0) TSK_HIP(hipEventRecord(b->done[q - 1], st));
    }
    for (size_t q = 1; q < G; ++q) TSK_HIP(hipStreamWaitEvent(s, b->done[q - 1], 0));
    return TSK_OK;
}

tsk_status kolmo_batch_set_inputs(KolmoBatch* b, const void* const* xbase, const int* jmax, hipStream_t s) {
    const size_t isz = b->fp32 ? sizeof(ColInst<float>) : sizeof(ColInst<double>);
    const size_t count = b->host_insts.size() / isz;
    for (size_t i = 0; i < count; ++i) {
        char* e = b->host_insts.data() + isz * i;
        if (b->fp32) {
            auto* c = reinterpret_cast<ColInst<float>*>(e);
            c->xbase = static_cast<const float*>(xbase[i]);
            c->jmax = jmax[i];
        } else {
            auto* c = reinterpret_cast<ColInst<double>*>(e);
            c->xbase = static_cast<const double*>(xbase[i]);
            c->jmax = jmax[i];
        }
    }
    TSK_HIP(hipMemcpyAsync(b->insts.ptr, b->host_insts.data(), b->host_insts.size(), hipMemcpyHostToDevice, s));
    // the host copy may be rewritten by the next call before this copy runs
    TSK_HIP(hipStreamSynchronize(s));
    return TSK_OK;
}

void kolmo_batch_free(KolmoBatch* b) { delete b; }

int kolmo_batch_groups(const KolmoBatch* b) { return int(b->groups.size()); }

}  // namespace tsk
