// Krylov-basis kernels of the Arnoldi driver: classical Gram-Schmidt applied
// twice (CGS2), norms, normalisation and Ritz vectors, for a batch of
// independent Arnoldi instances advancing in lockstep.
//
// Algorithm 1 (Sec. 3.2.1) projects the new matvec output w on the basis once,
// h = V^T w, f = w - V h; here the projection is repeated (h1 + h2), the usual
// cure for the loss of orthogonality of a single classical pass.  The operation
// is a tall-skinny matrix-vector product (one new vector per step), so every
// kernel streams V once with coalesced loads; sums are accumulated in FP64
// (complex128 for complex states) whatever the storage type of V.
//
// Work split: blockIdx.y selects the instance (its descriptor holds every
// pointer); blocks of kBT = 256 threads own contiguous chunks of kChunk = 256
// elements (small chunks keep enough workgroups busy at the 10^4-element
// states of the 128^2 grids).  A dot pass stages the chunk of w in LDS, then each of the four
// wavefronts takes every fourth basis vector, reads its chunk coalesced and
// reduces the 64 lane sums with cross-lane shuffles; several vectors' loads are
// in flight at once.  Per-block partial sums are
// reduced in a fixed order (lanes over blocks, then a shuffle tree) by one
// workgroup per instance, so results are bitwise reproducible run to run and
// independent of the batch composition.
#pragma once

#include "common.hpp"

namespace tsk {

constexpr int kBT = 256;
constexpr int kChunk = 256;
constexpr int kEPT = kChunk / kBT;

inline int cgs_blocks(int64_t n) { return int((n + kChunk - 1) / kChunk); }

// One Arnoldi instance, as seen by the device.  Scalars in `scal`:
// [0] ||x0||^2, [1] ||w before projection||^2, [2] beta; int flag at scal+32,
// int block counter of the fused normalisation at scal+34 (cgs_counter).
struct KryDesc {
    void* V;            // (m+1) vectors of the state type, stride ldv
    void* w;            // matvec output (state type)
    void* w64;          // FP64 / complex128 working copy of w
    double2* H;         // (m+1) x m complex128, column-major, leading dim ldh
    double2* partial;   // nblk x (m+1) partial dots
    double* pnrm;       // nblk partial squared norms
    double2* partial2;  // second buffers: a fused pass reads one and writes the other
    double* pnrm2;
    double2* h;         // m+1 reduced coefficients
    double* scal;       // 64 device scalars
    double2* Z;         // eigensolver scratch (p x p, standalone use)
    double2* S;         // eigenvectors of T (p x p)
    double2* Y;         // unit Ritz coordinates of the wanted pairs (p x k)
    double2* mu;        // Ritz values (p)
    double* res;        // residual estimates (p)
    int* sel;           // wanted indices (k)
    RitzResult* rr;
    const void* x0;     // start vector (state type)
    void* ritz;         // optional Ritz vectors, n x k complex128 (may be null)
    double* out;        // gathered outputs: mu (2k), lambda (2k), residual (k)
    int64_t ldv, n;
    const int* stop;    // optional host-written flag (pinned): the run no longer needs this instance's analyses
    int ldh, nblk;
    int active;         // 0: instance finished, kernels skip it
    int steps;          // Arnoldi steps taken (set before the output kernels)
    double dup_rel;     // duplicate width of the wanted-set rule (0 for FP64)
    double res_floor;   // relative residual floor: converged when res <= max(tol, res_floor |mu|)
    double T;           // sampling period (lambda = log(mu)/T)
    // Krylov-Schur contraction (k_ks_contract): kept-set rule and output
    double* ksW;        // m x p orthonormal rotation of the basis, column-major (ld m)
    double ks_delta;    // wanted when |mu| >= 1 - ks_delta
    int ks_pmax;        // largest order kept
    // step offset of the batched restart phase: an instance at order p_i expands
    // in lockstep with the others, its own step being the batch step + poff
    // (0 in ordinary runs); steps at or beyond order m = ldh - 1 are skipped
    int poff;
};

__host__ __device__ inline int* cgs_counter(const KryDesc& d) { return reinterpret_cast<int*>(d.scal + 34); }

// Host launchers; TS = double, float (real states) or double2 (complex).
// Grids: x over chunks of the longest instance, y over `count` instances.
template <typename TS>
void launch_check_finite(const KryDesc* D, int count, int64_t nmax, hipStream_t s);  // x0 -> scal+32
// Pass 1: partials of conj(V_i) . src and |src|^2, src = x0 (p = 0) or w.
template <typename TS>
void launch_dot(const KryDesc* D, int count, int nblk_max, int p, bool from_x0, hipStream_t s);
// scal[slot] = sum_b pnrm (the chunk norms of the last dot pass).
void launch_reduce_norm(const KryDesc* D, int count, int slot, hipStream_t s);
// Fused Gram-Schmidt pass (1 or 2) of step j with the previous reduction
// folded in, and the final normalisation with beta and the flags.
// fuse_final (pass 2): the last block of each instance also does the work of
// launch_scale_final, whose launch is then skipped (for short states, where a
// launch costs more than one block scaling the vector).
constexpr int kFuseFinalMaxBlocks = 64;
// Passes over more than this many chunks take their coefficients from one
// reduction launch (k_reduce_coefs) instead of every block reducing the
// partial dots itself.  Measured with interleaved runs of both forms: at 115
// chunks (256^2 states) the folded form saves the launch (256^2 solves FP64
// 6.06 -> 5.77 ms, FP32 8.23 -> 8.05 ms); with 255 chunks (384^2, in the
// 64-instance sweep) and 456 (512^2) the separate launch is faster (sweep 57
// against 64 ms with the threshold at 256 or 512).
constexpr int kPreReduceMinBlocks = 129;
template <typename TS>
void launch_cgs_pass(const KryDesc* D, int count, int nblk_max, int p, int j, int pass, bool fuse_final,
                     hipStream_t s, int pextra = 0);
template <typename TS>
void launch_scale_final(const KryDesc* D, int count, int64_t nmax, int j, hipStream_t s);
// V_{j+1} = w64 / beta (j >= 0), or V_0 = x0 / ||x0|| (j < 0).
template <typename TS>
void launch_scale(const KryDesc* D, int count, int64_t nmax, int j, hipStream_t s);
// ritz[s*n + e] = sum_i V_i[e] Y[s*p + i] for the nsel wanted pairs, p = steps.
template <typename TS>
void launch_ritz_vectors(const KryDesc* D, int count, int64_t nmax, int k, hipStream_t s);
// Krylov-Schur truncation of a real basis (TS = double or float): Vout_c =
// sum_{j<m} Vin_j W[j + m c] (c < kp), Vout_kp = Vin_m; Vin and Vout distinct.
template <typename TS>
void launch_rotate(const void* Vin, void* Vout, const double* W, int64_t n, int64_t ldv, int m, int kp, hipStream_t s);
// out: mu, lambda = log(mu)/T, residual of the wanted pairs.
void launch_gather(const KryDesc* D, int count, int k, hipStream_t s);

}  // namespace tsk
