// Learned start vector: a three-layer perceptron (Re, alpha) -> 32 x 32 block
// of low Fourier coefficients, its training (forward, backward, Adam), the
// training target made from Ritz vectors, and the start vector assembled from
// a prediction.  Not part of the paper: Algorithm 1 (Sec. 3.2.1) takes any
// start vector, and one close to the wanted invariant subspace shortens the
// Krylov sequence.
//
// Network: x = features(Re, alpha) in [-1, 1]^2 -> A1 = tanh(x W1 + b1)
// (W wide) -> A2 = tanh(A1 W2 + b2) -> Y = A2 W3 + b3 (2048).  Master weights,
// gradients and Adam moments are FP32; W2 and W3 also live as bfloat16 copies.
// The two large layers, their weight gradients and the back-propagated
// activations are products of bfloat16 operands (round to nearest even from
// FP32) accumulated in FP32 on the matrix cores: one MFMA GEMM kernel with
// transpose flags and fused epilogues (bias + tanh + bfloat16 copy; bias;
// tanh derivative + bfloat16 copy; plain store).  Layer 1 (two inputs), the
// loss, bias gradients and Adam are FP32 vector kernels.  Loss and bias sums
// are reduced in a fixed order, so a training run is reproducible bit for bit.
//
// Parameter vector layout (flat, FP32): W1 [2][W], b1 [W], W2 [W][W], b2 [W],
// W3 [W][2048], b3 [2048], weights row-major [in][out].
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ops.hpp"

namespace tsk {

namespace {

constexpr int kOut = 2048;
constexpr int kBjx = 32, kBjy0 = -16, kBny = 32;  // block jx in [0,32), jy in [-16,16)
constexpr int kSlots = kBjx * kBny;               // 1024 complex slots = kOut reals
static_assert(2 * kSlots == kOut, "block layout");
constexpr int kMaxBatch = 4096;

// ---- bfloat16 (raw bits) ----------------------------------------------------------
__device__ inline uint16_t f2bf(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return uint16_t((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}

// ---- GEMM: C[M x N] = op(A)[M x K] op(B)[K x N], bfloat16 in, FP32 accumulate ----
// op(A)(m, k) = A[m lda + k] (TA = false) or A[k lda + m] (TA = true);
// op(B)(k, n) = B[k ldb + n] (TB = false) or B[n ldb + k] (TB = true).
// Tile 64 x 64 per 256-thread workgroup, four wavefronts of 32 x 32, each as
// 2 x 2 MFMA 16x16x16 blocks; K advances in slices of 32 staged in LDS with
// k contiguous per row (A) and per column (B), zero-filled past the edges.
enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

struct GemmArgs {
    const uint16_t* A;
    const uint16_t* B;
    int M, N, K, lda, ldb, ldc;
    float* C;             // FP32 result
    uint16_t* Ch;         // bfloat16 copy (BIAS_TANH, DTANH; may be null)
    const float* bias;    // per column (BIAS, BIAS_TANH)
    const float* act;     // tanh activations, stride ldc (DTANH)
};

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int GT = 64, GK = 32, GLD = GK + 8;

// Split K: for products with a long K and few 64 x 64 tiles (the back-products of
// the output layer, K = 2048, eight tiles), grid z splits K into equal slabs;
// each workgroup stores its FP32 partial tile in a workspace and a second kernel
// sums the slabs in a fixed order and applies the epilogue, so the result does
// not depend on scheduling.
struct GemmSplit {
    float* part;  // [splits][M][N] partial products (null: no split)
    int kslab;    // K per slab (a multiple of GK)
};

template <int EPI>
__device__ inline void gemm_epilogue(const GemmArgs& g, int row, int col, float v) {
    const size_t o = size_t(row) * g.ldc + col;
    if constexpr (EPI == EPI_BIAS) v += g.bias[col];
    if constexpr (EPI == EPI_BIAS_TANH) v = tanhf(v + g.bias[col]);
    if constexpr (EPI == EPI_DTANH) {
        const float a = g.act[o];
        v = v * (1.0f - a * a);
    }
    g.C[o] = v;
    if constexpr (EPI == EPI_BIAS_TANH || EPI == EPI_DTANH)
        if (g.Ch) g.Ch[o] = f2bf(v);
}

// Operands whose k index is contiguous (A with TA = false, B with TB = true) are
// read as 16-byte vectors of 8 bfloat16 (one per thread per K slice); the others
// element by element.  The next slice's global loads are issued before the
// current slice's products, so they overlap.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g, GemmSplit sp) {
    __shared__ __align__(16) uint16_t As[GT * GLD];
    __shared__ __align__(16) uint16_t Bs[GT * GLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kbeg = sp.part ? int(blockIdx.z) * sp.kslab : 0;
    const int kend = sp.part ? min(g.K, kbeg + sp.kslab) : g.K;
    // 16-byte loads need 16-byte aligned rows (k0 is a multiple of 8)
    const bool avec = ((reinterpret_cast<uintptr_t>(g.A) | (uintptr_t(g.lda) * 2)) & 15) == 0;
    const bool bvec = ((reinterpret_cast<uintptr_t>(g.B) | (uintptr_t(g.ldb) * 2)) & 15) == 0;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    // staging registers of one K slice
    typedef unsigned short v8u __attribute__((ext_vector_type(8)));
    v8u av{}, bv{};
    uint16_t as8[8], bs8[8];
    auto load = [&](int k0) {
        if constexpr (!TA) {
            // A[m][k]: thread -> row tid/4, k chunk 8 (tid % 4)
            const int m = m0 + (tid >> 2), k = k0 + 8 * (tid & 3);
            if (m < g.M && k + 8 <= g.K && avec) {
                av = *reinterpret_cast<const v8u*>(g.A + size_t(m) * g.lda + k);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) av[e] = (m < g.M && k + e < g.K) ? g.A[size_t(m) * g.lda + k + e] : 0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int mm = tid & 63, kk = (tid >> 6) + 4 * i;
                const int m = m0 + mm, k = k0 + kk;
                as8[i] = (m < g.M && k < g.K) ? g.A[size_t(k) * g.lda + m] : 0;
            }
        }
        if constexpr (TB) {
            const int n = n0 + (tid >> 2), k = k0 + 8 * (tid & 3);
            if (n < g.N && k + 8 <= g.K && bvec) {
                bv = *reinterpret_cast<const v8u*>(g.B + size_t(n) * g.ldb + k);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = (n < g.N && k + e < g.K) ? g.B[size_t(n) * g.ldb + k + e] : 0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int nn = tid & 63, kk = (tid >> 6) + 4 * i;
                const int n = n0 + nn, k = k0 + kk;
                bs8[i] = (n < g.N && k < g.K) ? g.B[size_t(k) * g.ldb + n] : 0;
            }
        }
    };
    auto stage = [&]() {
        if constexpr (!TA) {
            *reinterpret_cast<v8u*>(&As[(tid >> 2) * GLD + 8 * (tid & 3)]) = av;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) As[(tid & 63) * GLD + (tid >> 6) + 4 * i] = as8[i];
        }
        if constexpr (TB) {
            *reinterpret_cast<v8u*>(&Bs[(tid >> 2) * GLD + 8 * (tid & 3)]) = bv;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(tid & 63) * GLD + (tid >> 6) + 4 * i] = bs8[i];
        }
    };
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        stage();
        __syncthreads();
        if (k0 + GK < kend) load(k0 + GK);  // in flight during the products below
#pragma unroll
        for (int ks = 0; ks < GK; ks += 16) {
            v4s a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = *reinterpret_cast<const v4s*>(&As[(wm + 16 * t + (lane & 15)) * GLD + ks + 4 * (lane >> 4)]);
                b[t] = *reinterpret_cast<const v4s*>(&Bs[(wn + 16 * t + (lane & 15)) * GLD + ks + 4 * (lane >> 4)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // D layout of the 16x16 block: lane holds column lane % 16, rows 4 (lane / 16) + r.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int col = n0 + wn + 16 * j + (lane & 15);
                if (row >= g.M || col >= g.N) continue;
                if (sp.part)
                    sp.part[(size_t(blockIdx.z) * g.M + row) * g.N + col] = acc[i][j][r];
                else
                    gemm_epilogue<EPI>(g, row, col, acc[i][j][r]);
            }
}

// Sum of the split-K slabs in slab order, then the epilogue.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g, const float* __restrict__ part, int splits) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= int64_t(g.M) * g.N) return;
    float v = 0.0f;
    for (int z = 0; z < splits; ++z) v += part[size_t(z) * g.M * g.N + e];
    gemm_epilogue<EPI>(g, int(e / g.N), int(e % g.N), v);
}

// Split K when the tile grid is small (< 64 workgroups) and K long: slabs of at
// least 128, as many as bring the grid to about 128 workgroups.
inline int gemm_splits(int M, int N, int K) {
    const int tiles = ((M + GT - 1) / GT) * ((N + GT - 1) / GT);
    if (tiles >= 64 || K < 512) return 1;
    int s = 1;
    while (tiles * s * 2 <= 128 && K / (s * 2) >= 128) s *= 2;
    return s;
}

template <bool TA, bool TB, int EPI>
void gemm(const GemmArgs& g, float* work, hipStream_t s) {
    const int splits = work ? gemm_splits(g.M, g.N, g.K) : 1;
    GemmSplit sp{nullptr, g.K};
    if (splits > 1) {
        sp.part = work;
        sp.kslab = ((g.K + splits - 1) / splits + GK - 1) / GK * GK;
    }
    dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, splits);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, g, sp);
    if (splits > 1) {
        const int64_t ne = int64_t(g.M) * g.N;
        hipLaunchKernelGGL(k_gemm_reduce<EPI>, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, g, work, splits);
    }
}

// ---- vector kernels -------------------------------------------------------------------
// Layer 1: x = (p - lo) * sc - 1 per input, A1 = tanh(x W1 + b1).
__global__ void k_l1_fwd(const float* __restrict__ in, int B, int W, const float* __restrict__ w,
                         float lo0, float sc0, float lo1, float sc1, float* __restrict__ X,
                         float* __restrict__ A1, uint16_t* __restrict__ A1h) {
    const float* W1 = w;
    const float* b1 = w + 2 * W;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < B * W; e += gridDim.x * blockDim.x) {
        const int b = e / W, n = e - b * W;
        const float x0 = (in[2 * b] - lo0) * sc0 - 1.0f;
        const float x1 = (in[2 * b + 1] - lo1) * sc1 - 1.0f;
        if (n == 0) {
            X[2 * b] = x0;
            X[2 * b + 1] = x1;
        }
        const float a = tanhf(x0 * W1[n] + x1 * W1[W + n] + b1[n]);
        A1[e] = a;
        A1h[e] = f2bf(a);
    }
}

constexpr int kLossBlocks = 64;

// dY = scale (Y - T); per-block partial sums of (Y - T)^2 in FP64.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ Y, const float* __restrict__ T,
                                              int64_t count, float scale, float* __restrict__ dY,
                                              uint16_t* __restrict__ dYh, double* __restrict__ partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x) {
        const float d = Y[e] - T[e];
        acc += double(d) * double(d);
        const float gd = scale * d;
        dY[e] = gd;
        dYh[e] = f2bf(gd);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const double* __restrict__ partial, int nb, double inv_count, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += partial[i];
        *out = s * inv_count;
    }
}

// g[n] = sum_b D[b][n] (FP64 accumulation, rows in order).  Rows are loaded
// eight at a time ahead of the additions (the sum stays in row order), so the
// loads overlap instead of each waiting for the previous addition.
__global__ void k_colsum(const float* __restrict__ D, int B, int N, float* __restrict__ g) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= B; b += 8) {
        float d[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) d[i] = D[size_t(b + i) * N + n];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += d[i];
    }
    for (; b < B; ++b) s += D[size_t(b) * N + n];
    g[n] = float(s);
}

// gW1[i][n] = sum_b X[b][i] dZ1[b][n], gb1[n] = sum_b dZ1[b][n] (rows in order,
// loaded eight at a time as in k_colsum).
__global__ void k_l1_grad(const float* __restrict__ X, const float* __restrict__ dZ1, int B, int W,
                          float* __restrict__ grad) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= W) return;
    double s0 = 0.0, s1 = 0.0, sb = 0.0;
    int b = 0;
    for (; b + 8 <= B; b += 8) {
        float d[8], x0[8], x1[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            d[i] = dZ1[size_t(b + i) * W + n];
            x0[i] = X[2 * (b + i)];
            x1[i] = X[2 * (b + i) + 1];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            s0 += double(x0[i]) * double(d[i]);
            s1 += double(x1[i]) * double(d[i]);
            sb += double(d[i]);
        }
    }
    for (; b < B; ++b) {
        const double d = dZ1[size_t(b) * W + n];
        s0 += double(X[2 * b]) * d;
        s1 += double(X[2 * b + 1]) * d;
        sb += d;
    }
    grad[n] = float(s0);
    grad[W + n] = float(s1);
    grad[2 * W + n] = float(sb);
}

// Adam (Kingma & Ba 2015) with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t);
// refreshes the bfloat16 copy.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                       float c2, uint16_t* __restrict__ wh) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.0f - b1) * ge;
        const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        const float we = w[e] - lr * (me * c1) / (sqrtf(ve * c2) + eps);
        w[e] = we;
        wh[e] = f2bf(we);
    }
}

__global__ void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wh, int64_t count) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x)
        wh[e] = f2bf(w[e]);
}

// Xavier-uniform weights from splitmix64 output e (flat index), zero biases.
__global__ void k_init(float* __restrict__ w, int W, uint64_t seed, float lim1, float lim2, float lim3) {
    const int64_t o_b1 = 2 * int64_t(W), o_W2 = 3 * int64_t(W), o_b2 = o_W2 + int64_t(W) * W;
    const int64_t o_W3 = o_b2 + W, o_b3 = o_W3 + int64_t(W) * kOut, total = o_b3 + kOut;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
        float lim = 0.0f;
        if (e < o_b1) lim = lim1;
        else if (e >= o_W2 && e < o_b2) lim = lim2;
        else if (e >= o_W3 && e < o_b3) lim = lim3;
        if (lim == 0.0f) {
            w[e] = 0.0f;
            continue;
        }
        const double u = double(splitmix_at(seed, uint64_t(e)) >> 11) * 0x1.0p-53;
        w[e] = float(double(lim) * (2.0 * u - 1.0));
    }
}

// ---- block <-> packed spectral state --------------------------------------------------
// Packed complex coefficient c of the Navier-Stokes state: c < M is (0, c+1);
// otherwise c - M = (jx-1)(2M+1) + (jy+M).  Slot s of the block is
// (jx, jy) = (s / 32, s % 32 - 16).
__device__ inline int64_t slot_to_coef(int s, int M) {
    const int jx = s / kBny, jy = s % kBny + kBjy0;
    if (jx == 0) return (jy >= 1 && jy <= M) ? jy - 1 : -1;
    if (jx > M || jy < -M || jy > M) return -1;
    return int64_t(M) + int64_t(jx - 1) * (2 * M + 1) + (jy + M);
}

__device__ inline double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline int block_min_int(int v, int* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const int r = red[0];
    __syncthreads();
    return r;
}

constexpr int kTB = 256;
constexpr int kSPT = kSlots / kTB;  // slots per thread
constexpr double kTie = 1e-6;

// Training target from k Ritz vectors Z (vector-major, n complex128 each).  One
// workgroup.  Per used vector: part = Re or Im (larger norm); block
// coefficients; pivot = smallest slot with |c|^2 >= (1 - kTie) max; rotate by
// the x-translation (jx_p > 0) or sign (jx_p = 0) that makes the pivot real
// positive; add the unit-norm block.  Output: the sum scaled to unit norm.
__global__ __launch_bounds__(kTB) void k_ritz_target(const double2* __restrict__ Z, int64_t n, int k,
                                                     uint64_t use_lo, uint64_t use_hi, int M,
                                                     float* __restrict__ out) {
    __shared__ double red[kTB];
    __shared__ int redi[kTB];
    double2 acc[kSPT];
#pragma unroll
    for (int q = 0; q < kSPT; ++q) acc[q] = cmk<double2>(0.0, 0.0);
    for (int s = 0; s < k; ++s) {
        const bool use = s < 64 ? ((use_lo >> s) & 1ull) : ((use_hi >> (s - 64)) & 1ull);
        if (!use) continue;
        const double2* z = Z + size_t(s) * n;
        double nr = 0.0, ni = 0.0;
        for (int64_t e = threadIdx.x; e < n; e += kTB) {
            const double2 v = z[e];
            nr += v.x * v.x;
            ni += v.y * v.y;
        }
        nr = block_sum(nr, red);
        ni = block_sum(ni, red);
        const bool im = ni > nr;
        double2 c[kSPT];
        double mag[kSPT];
        double mmax = 0.0, bn = 0.0;
#pragma unroll
        for (int q = 0; q < kSPT; ++q) {
            const int sl = threadIdx.x + q * kTB;
            const int64_t p = slot_to_coef(sl, M);
            c[q] = cmk<double2>(0.0, 0.0);
            if (p >= 0) {
                const double2 a = z[2 * p], b = z[2 * p + 1];
                c[q] = im ? cmk<double2>(a.y, b.y) : cmk<double2>(a.x, b.x);
            }
            mag[q] = c[q].x * c[q].x + c[q].y * c[q].y;
            mmax = fmax(mmax, mag[q]);
            bn += mag[q];
        }
        mmax = block_max(mmax, red);
        bn = block_sum(bn, red);
        if (!(mmax > 0.0)) continue;
        int piv = kSlots;
#pragma unroll
        for (int q = 0; q < kSPT; ++q) {
            const int sl = threadIdx.x + q * kTB;
            if (mag[q] >= (1.0 - kTie) * mmax && sl < piv) piv = sl;
        }
        piv = block_min_int(piv, redi);
        // pivot coefficient, broadcast through LDS by its owner
        if (threadIdx.x == (piv % kTB)) {
            const double2 cp = c[piv / kTB];
            red[0] = cp.x;
            red[1] = cp.y;
        }
        __syncthreads();
        const double cpx = red[0], cpy = red[1];
        __syncthreads();
        const int jp = piv / kBny;
        const double phi = atan2(cpy, cpx);
        const double inv = 1.0 / sqrt(bn);
#pragma unroll
        for (int q = 0; q < kSPT; ++q) {
            const int sl = threadIdx.x + q * kTB;
            const int jx = sl / kBny;
            double2 r;
            if (jp > 0) {
                double sn, cs;
                sincos(-double(jx) * phi / double(jp), &sn, &cs);
                r = cmk<double2>(cs, sn);
            } else {
                r = cmk<double2>(cpx >= 0.0 ? 1.0 : -1.0, 0.0);
            }
            const double2 v = cmul(r, c[q]);
            acc[q].x += v.x * inv;
            acc[q].y += v.y * inv;
        }
    }
    double an = 0.0;
#pragma unroll
    for (int q = 0; q < kSPT; ++q) an += acc[q].x * acc[q].x + acc[q].y * acc[q].y;
    an = block_sum(an, red);
    const double sc = an > 0.0 ? 1.0 / sqrt(an) : 0.0;
#pragma unroll
    for (int q = 0; q < kSPT; ++q) {
        const int sl = threadIdx.x + q * kTB;
        out[2 * sl] = float(acc[q].x * sc);
        out[2 * sl + 1] = float(acc[q].y * sc);
    }
}

// Norms for the start vector: nrm[0] = ||p||^2 (prediction scattered to the
// state; NaN propagates), nrm[1] = ||r||^2.  One workgroup.
template <typename TS>
__global__ __launch_bounds__(kTB) void k_decode_norms(const float* __restrict__ y, const TS* __restrict__ r,
                                                      int64_t n, int M, double* __restrict__ nrm) {
    __shared__ double red[kTB];
    double pp = 0.0, rr = 0.0;
    for (int sl = threadIdx.x; sl < kSlots; sl += kTB) {
        if (slot_to_coef(sl, M) < 0) continue;
        const double a = y[2 * sl], b = y[2 * sl + 1];
        pp += a * a + b * b;
    }
    for (int64_t e = threadIdx.x; e < n; e += kTB) {
        const double v = double(r[e]);
        rr += v * v;
    }
    pp = block_sum(pp, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        nrm[0] = pp;
        nrm[1] = rr;
    }
}

// v0 = p / ||p|| + gamma r / ||r||, or r / ||r|| when ||p|| is zero or not finite.
template <typename TS>
__global__ void k_decode(const float* __restrict__ y, const TS* __restrict__ r, int64_t n, int M, double gamma,
                         const double* __restrict__ nrm, TS* __restrict__ v0) {
    const double pp = nrm[0], rr = nrm[1];
    const bool use = pp > 0.0 && pp <= 1.0e300;  // false for NaN and Inf
    const double ip = use ? 1.0 / sqrt(pp) : 0.0;
    const double ir = rr > 0.0 ? 1.0 / sqrt(rr) : 0.0;
    const double gr = use ? gamma * ir : ir;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        // inverse of slot_to_coef for the coefficient e / 2
        const int64_t c = e >> 1;
        int jx, jy;
        if (c < M) {
            jx = 0;
            jy = int(c) + 1;
        } else {
            const int64_t q = c - M;
            jx = int(q / (2 * M + 1)) + 1;
            jy = int(q % (2 * M + 1)) - M;
        }
        double p = 0.0;
        if (use && jx < kBjx && jy >= kBjy0 && jy < kBjy0 + kBny)
            p = y[2 * (jx * kBny + (jy - kBjy0)) + (e & 1)];
        v0[e] = TS(p * ip + gr * double(r[e]));
    }
}

int grid_for(int64_t count, int cap = 2048) {
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return int(g);
}

}  // namespace

// ---- the network object -----------------------------------------------------------------
struct Mlp {
    int W = 0;
    hipStream_t stream = nullptr;
    double lo[2] = {0, 0}, hi[2] = {1, 1};
    int64_t np = 0;
    int64_t o_W1 = 0, o_b1 = 0, o_W2 = 0, o_b2 = 0, o_W3 = 0, o_b3 = 0;
    DevBuf w, wh, g, m, v;
    DevBuf in1, X, A1, A1h, A2, A2h, Y, dY, dYh, dZ2, dZ2h, dZ1, partial, loss, nrm;
    DevBuf gwork;  // split-K partial products
    int cap = 0;
    int64_t t = 0;
    bool has_params = false;

    tsk_status init_layout() {
        o_W1 = 0;
        o_b1 = 2 * int64_t(W);
        o_W2 = o_b1 + W;
        o_b2 = o_W2 + int64_t(W) * W;
        o_W3 = o_b2 + W;
        o_b3 = o_W3 + int64_t(W) * kOut;
        np = o_b3 + kOut;
        TSK_TRY(w.ensure(size_t(np) * 4));
        TSK_TRY(wh.ensure(size_t(np) * 2));
        TSK_TRY(g.ensure(size_t(np) * 4));
        TSK_TRY(m.ensure(size_t(np) * 4));
        TSK_TRY(v.ensure(size_t(np) * 4));
        TSK_TRY(partial.ensure(kLossBlocks * 8));
        TSK_TRY(nrm.ensure(64));
        TSK_TRY(in1.ensure(64));
        return TSK_OK;
    }
    tsk_status reserve(int B, int loss_slots) {
        if (B > cap) {
            TSK_TRY(X.ensure(size_t(B) * 2 * 4));
            TSK_TRY(A1.ensure(size_t(B) * W * 4));
            TSK_TRY(A1h.ensure(size_t(B) * W * 2));
            TSK_TRY(A2.ensure(size_t(B) * W * 4));
            TSK_TRY(A2h.ensure(size_t(B) * W * 2));
            TSK_TRY(Y.ensure(size_t(B) * kOut * 4));
            TSK_TRY(dY.ensure(size_t(B) * kOut * 4));
            TSK_TRY(dYh.ensure(size_t(B) * kOut * 2));
            TSK_TRY(dZ2.ensure(size_t(B) * W * 4));
            TSK_TRY(dZ2h.ensure(size_t(B) * W * 2));
            TSK_TRY(dZ1.ensure(size_t(B) * W * 4));
            cap = B;
        }
        // the largest split-K workspace of the six products at this batch (not
        // monotone in B: a larger batch may take fewer slabs)
        size_t wf = 0;
        const int shapes[6][3] = {{B, W, W}, {B, kOut, W}, {W, kOut, B}, {B, W, kOut}, {W, W, B}, {B, W, W}};
        for (const auto& sh : shapes) {
            const int sp = gemm_splits(sh[0], sh[1], sh[2]);
            if (sp > 1) wf = std::max(wf, size_t(sp) * sh[0] * sh[1]);
        }
        TSK_TRY(gwork.ensure(std::max<size_t>(wf, 1) * 4));
        TSK_TRY(loss.ensure(size_t(loss_slots < 1 ? 1 : loss_slots) * 8));
        return TSK_OK;
    }
    float* wf() const { return w.as<float>(); }
    const uint16_t* whp(int64_t off) const { return wh.as<uint16_t>() + off; }

    // Forward pass; Y (B x 2048) lands in `out` (may be the internal Y buffer).
    void forward(const float* in, int B, float* out, hipStream_t s) {
        const float sc0 = float(2.0 / (hi[0] - lo[0])), sc1 = float(2.0 / (hi[1] - lo[1]));
        hipLaunchKernelGGL(k_l1_fwd, dim3(grid_for(int64_t(B) * W)), dim3(256), 0, s, in, B, W, wf(), float(lo[0]),
                           sc0, float(lo[1]), sc1, X.as<float>(), A1.as<float>(), A1h.as<uint16_t>());
        GemmArgs a{};
        a.A = A1h.as<uint16_t>(); a.B = whp(o_W2); a.M = B; a.N = W; a.K = W;
        a.lda = W; a.ldb = W; a.ldc = W; a.C = A2.as<float>(); a.Ch = A2h.as<uint16_t>(); a.bias = wf() + o_b2;
        gemm<false, false, EPI_BIAS_TANH>(a, gwork.as<float>(), s);
        GemmArgs b{};
        b.A = A2h.as<uint16_t>(); b.B = whp(o_W3); b.M = B; b.N = kOut; b.K = W;
        b.lda = W; b.ldb = kOut; b.ldc = kOut; b.C = out; b.bias = wf() + o_b3;
        gemm<false, false, EPI_BIAS>(b, gwork.as<float>(), s);
    }

    // Loss into loss[slot] and the full gradient into g.
    void backward(const float* target, int B, int slot, hipStream_t s) {
        const int64_t cnt = int64_t(B) * kOut;
        hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, s, Y.as<float>(), target, cnt,
                           float(2.0 / double(cnt)), dY.as<float>(), dYh.as<uint16_t>(), partial.as<double>());
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, partial.as<double>(), kLossBlocks,
                           1.0 / double(cnt), loss.as<double>() + slot);
        float* G = g.as<float>();
        GemmArgs g3{};  // gW3 = A2h^T dYh
        g3.A = A2h.as<uint16_t>(); g3.B = dYh.as<uint16_t>(); g3.M = W; g3.N = kOut; g3.K = B;
        g3.lda = W; g3.ldb = kOut; g3.ldc = kOut; g3.C = G + o_W3;
        gemm<true, false, EPI_STORE>(g3, gwork.as<float>(), s);
        hipLaunchKernelGGL(k_colsum, dim3((kOut + 63) / 64), dim3(64), 0, s, dY.as<float>(), B, kOut, G + o_b3);
        GemmArgs d2{};  // dZ2 = (dYh W3h^T) * (1 - A2^2)
        d2.A = dYh.as<uint16_t>(); d2.B = whp(o_W3); d2.M = B; d2.N = W; d2.K = kOut;
        d2.lda = kOut; d2.ldb = kOut; d2.ldc = W; d2.C = dZ2.as<float>(); d2.Ch = dZ2h.as<uint16_t>();
        d2.act = A2.as<float>();
        gemm<false, true, EPI_DTANH>(d2, gwork.as<float>(), s);
        GemmArgs g2{};  // gW2 = A1h^T dZ2h
        g2.A = A1h.as<uint16_t>(); g2.B = dZ2h.as<uint16_t>(); g2.M = W; g2.N = W; g2.K = B;
        g2.lda = W; g2.ldb = W; g2.ldc = W; g2.C = G + o_W2;
        gemm<true, false, EPI_STORE>(g2, gwork.as<float>(), s);
        hipLaunchKernelGGL(k_colsum, dim3((W + 63) / 64), dim3(64), 0, s, dZ2.as<float>(), B, W, G + o_b2);
        GemmArgs d1{};  // dZ1 = (dZ2h W2h^T) * (1 - A1^2)
        d1.A = dZ2h.as<uint16_t>(); d1.B = whp(o_W2); d1.M = B; d1.N = W; d1.K = W;
        d1.lda = W; d1.ldb = W; d1.ldc = W; d1.C = dZ1.as<float>(); d1.act = A1.as<float>();
        gemm<false, true, EPI_DTANH>(d1, gwork.as<float>(), s);
        hipLaunchKernelGGL(k_l1_grad, dim3((W + 63) / 64), dim3(64), 0, s, X.as<float>(), dZ1.as<float>(), B, W,
                           G + o_W1);
    }

    void adam(double lr, hipStream_t s) {
        ++t;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = float(1.0 / (1.0 - std::pow(b1, double(t))));
        const float c2 = float(1.0 / (1.0 - std::pow(b2, double(t))));
        hipLaunchKernelGGL(k_adam, dim3(grid_for(np)), dim3(256), 0, s, wf(), g.as<float>(), m.as<float>(),
                           v.as<float>(), np, float(lr), float(b1), float(b2), 1e-8f, c1, c2, wh.as<uint16_t>());
    }

    tsk_status reset_optimizer() {
        TSK_HIP(hipMemsetAsync(m.ptr, 0, size_t(np) * 4, stream));
        TSK_HIP(hipMemsetAsync(v.ptr, 0, size_t(np) * 4, stream));
        hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(np)), dim3(256), 0, stream, wf(), wh.as<uint16_t>(), np);
        TSK_HIP(hipGetLastError());
        t = 0;
        has_params = true;
        return TSK_OK;
    }
};

tsk_status mlp_create(int width, const double* lo, const double* hi, hipStream_t s, Mlp** out) {
    if (width < 16 || width > 2048 || width % 16 != 0)
        return fail(TSK_EINVAL, "width must be a multiple of 16 in [16, 2048]");
    for (int i = 0; i < 2; ++i)
        if (!(hi[i] > lo[i]) || !std::isfinite(lo[i]) || !std::isfinite(hi[i]))
            return fail(TSK_EINVAL, "input box needs finite lo < hi");
    auto* n = new Mlp;
    n->W = width;
    n->stream = s;
    n->lo[0] = lo[0]; n->lo[1] = lo[1];
    n->hi[0] = hi[0]; n->hi[1] = hi[1];
    tsk_status st = n->init_layout();
    if (st < 0) {
        delete n;
        return st;
    }
    *out = n;
    return TSK_OK;
}

void mlp_free(Mlp* n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    delete n;
}

int64_t mlp_param_count(const Mlp* n) { return n->np; }

tsk_status mlp_init(Mlp* n, uint64_t seed) {
    auto lim = [](int a, int b) { return float(std::sqrt(6.0 / double(a + b))); };
    hipLaunchKernelGGL(k_init, dim3(grid_for(n->np)), dim3(256), 0, n->stream, n->wf(), n->W, seed, lim(2, n->W),
                       lim(n->W, n->W), lim(n->W, kOut));
    TSK_HIP(hipGetLastError());
    return n->reset_optimizer();
}

tsk_status mlp_set_params(Mlp* n, const float* host) {
    TSK_HIP(hipMemcpyAsync(n->w.ptr, host, size_t(n->np) * 4, hipMemcpyHostToDevice, n->stream));
    TSK_TRY(n->reset_optimizer());
    TSK_HIP(hipStreamSynchronize(n->stream));
    return TSK_OK;
}

tsk_status mlp_get_params(Mlp* n, float* host) {
    TSK_HIP(hipMemcpyAsync(host, n->w.ptr, size_t(n->np) * 4, hipMemcpyDeviceToHost, n->stream));
    TSK_HIP(hipStreamSynchronize(n->stream));
    return TSK_OK;
}

static tsk_status check_batch(const Mlp* n, int B) {
    if (!n->has_params) return fail(TSK_ESTATE, "network parameters not set (tsk_mlp_init or tsk_mlp_set_params)");
    if (B < 1 || B > kMaxBatch) return fail(TSK_EINVAL, "batch must be in [1, 4096]");
    return TSK_OK;
}

tsk_status mlp_forward(Mlp* n, const float* in, int B, float* out) {
    TSK_TRY(check_batch(n, B));
    TSK_TRY(n->reserve(B, 1));
    n->forward(in, B, out, n->stream);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status mlp_gradients(Mlp* n, const float* in, const float* target, int B, float* grad, double* loss_host) {
    TSK_TRY(check_batch(n, B));
    TSK_TRY(n->reserve(B, 1));
    n->forward(in, B, n->Y.as<float>(), n->stream);
    n->backward(target, B, 0, n->stream);
    TSK_HIP(hipGetLastError());
    if (grad) TSK_HIP(hipMemcpyAsync(grad, n->g.ptr, size_t(n->np) * 4, hipMemcpyDeviceToDevice, n->stream));
    if (loss_host) TSK_HIP(hipMemcpyAsync(loss_host, n->loss.ptr, 8, hipMemcpyDeviceToHost, n->stream));
    TSK_HIP(hipStreamSynchronize(n->stream));
    return TSK_OK;
}

tsk_status mlp_train(Mlp* n, const float* in, const float* target, int B, int steps, double lr, double* loss_host) {
    TSK_TRY(check_batch(n, B));
    if (steps < 1 || steps > 1000000) return fail(TSK_EINVAL, "steps must be in [1, 1e6]");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(TSK_EINVAL, "learning rate must be positive");
    TSK_TRY(n->reserve(B, steps));
    for (int i = 0; i < steps; ++i) {
        n->forward(in, B, n->Y.as<float>(), n->stream);
        n->backward(target, B, i, n->stream);
        n->adam(lr, n->stream);
    }
    TSK_HIP(hipGetLastError());
    if (loss_host)
        TSK_HIP(hipMemcpyAsync(loss_host, n->loss.ptr, size_t(steps) * 8, hipMemcpyDeviceToHost, n->stream));
    TSK_HIP(hipStreamSynchronize(n->stream));
    return TSK_OK;
}

tsk_status ritz_block_target(Operator* op, const void* ritz, int k, const int* use, float* target) {
    const int M = kolmo_cutoff(op);
    if (M < 0) return fail(TSK_EINVAL, "the block target needs a Navier-Stokes operator");
    if (k < 1 || k > 128) return fail(TSK_EINVAL, "k must be in [1, 128]");
    uint64_t lo = 0, hi = 0;
    for (int s = 0; s < k; ++s)
        if (!use || use[s]) (s < 64 ? lo : hi) |= 1ull << (s & 63);
    hipLaunchKernelGGL(k_ritz_target, dim3(1), dim3(kTB), 0, op->stream, static_cast<const double2*>(ritz), op->n, k,
                       lo, hi, M, target);
    TSK_HIP(hipGetLastError());
    TSK_HIP(hipStreamSynchronize(op->stream));
    return TSK_OK;
}

tsk_status mlp_start(Mlp* n, Operator* op, double Re, double alpha, double gamma, uint64_t seed, void* v0,
                     int* used) {
    const int M = kolmo_cutoff(op);
    if (M < 0) return fail(TSK_EINVAL, "the learned start needs a Navier-Stokes operator");
    if (!n->has_params) return fail(TSK_ESTATE, "network parameters not set");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(TSK_EINVAL, "gamma must be finite and >= 0");
    if (!std::isfinite(Re) || !std::isfinite(alpha)) return fail(TSK_EINVAL, "Re and alpha must be finite");
    const hipStream_t s = op->stream;
    TSK_HIP(hipStreamSynchronize(n->stream));  // training or parameter uploads done
    TSK_TRY(n->reserve(1, 1));
    // random part: iid N(0,1) physical field of `seed`, projected on the state space
    const int64_t pr = op->physical_reals();
    TSK_TRY(op->aw.phys.ensure(size_t(pr) * 8));
    TSK_TRY(op->aw.w.ensure(op->state_bytes()));
    TSK_TRY(normal_fill(op->aw.phys.as<double>(), pr, seed, s));
    if (op->kind == StateKind::Real32) TSK_TRY(narrow_to_float(op->aw.phys.as<double>(), op->aw.phys.as<float>(), pr, s));
    TSK_TRY(op->from_physical(op->aw.phys.ptr, op->aw.w.ptr));
    // prediction for (Re, alpha)
    const float in[2] = {float(Re), float(alpha)};
    TSK_HIP(hipMemcpyAsync(n->in1.ptr, in, sizeof(in), hipMemcpyHostToDevice, s));
    n->forward(n->in1.as<float>(), 1, n->Y.as<float>(), s);
    double* nrm = n->nrm.as<double>();
    const int64_t nn = op->n;
    if (op->kind == StateKind::Real32) {
        hipLaunchKernelGGL(k_decode_norms<float>, dim3(1), dim3(kTB), 0, s, n->Y.as<float>(), op->aw.w.as<float>(), nn,
                           M, nrm);
        hipLaunchKernelGGL(k_decode<float>, dim3(grid_for(nn)), dim3(256), 0, s, n->Y.as<float>(),
                           op->aw.w.as<float>(), nn, M, gamma, nrm, static_cast<float*>(v0));
    } else {
        hipLaunchKernelGGL(k_decode_norms<double>, dim3(1), dim3(kTB), 0, s, n->Y.as<float>(), op->aw.w.as<double>(),
                           nn, M, nrm);
        hipLaunchKernelGGL(k_decode<double>, dim3(grid_for(nn)), dim3(256), 0, s, n->Y.as<float>(),
                           op->aw.w.as<double>(), nn, M, gamma, nrm, static_cast<double*>(v0));
    }
    TSK_HIP(hipGetLastError());
    double h[2];
    TSK_HIP(hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    if (used) *used = (h[0] > 0.0 && h[0] <= 1.0e300) ? 1 : 0;
    return TSK_OK;
}

}  // namespace tsk
