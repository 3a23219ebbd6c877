// Krylov-basis kernels of the Arnoldi driver: classical Gram-Schmidt applied
// twice (CGS2), norms, normalisation and Ritz vectors.
//
// Algorithm 1 (Sec. 3.2.1) projects the new matvec output w on the basis once,
// h = V^T w, f = w - V h; here the projection is repeated (h1 + h2), the usual
// cure for the loss of orthogonality of a single classical pass.  The operation
// is a tall-skinny matrix-vector product (one new vector per step), so every
// kernel streams V once with coalesced loads; sums are accumulated in FP64
// (complex128 for complex states) whatever the storage type of V.
//
// Work split: blocks of kBT = 256 threads own contiguous chunks of kChunk = 1024
// elements.  A dot pass stages the chunk of w in LDS, then each of the four
// wavefronts takes every fourth basis vector, reads its chunk coalesced and
// reduces the 64 lane sums with cross-lane shuffles.  Per-block partial sums are
// reduced in a fixed order by a one-block kernel, so results are bitwise
// reproducible run to run.
#pragma once

#include "common.hpp"

namespace tsk {

constexpr int kBT = 256;
constexpr int kChunk = 1024;
constexpr int kEPT = kChunk / kBT;

inline int cgs_blocks(int64_t n) { return int((n + kChunk - 1) / kChunk); }

// Host launchers; TS = double, float (real states) or double2 (complex).
// Pass 1: partial[b*p + i] = sum_chunk conj(V_i) w ; pnrm[b] = sum_chunk |w|^2.
template <typename TS>
void launch_dot(const TS* V, int64_t ldv, int p, const TS* w, int64_t n, double2* partial, double* pnrm,
                hipStream_t s);
// Reduce partials: h[i] = sum_b partial[b*p+i]; Hcol[i] = (first ? 0 : Hcol[i]) + h[i];
// scal[slot] = sum_b pnrm[b] when pnrm != null.
void launch_reduce(const double2* partial, int nblk, int p, double2* h, double2* Hcol, int first,
                   const double* pnrm, double* scal, int slot, hipStream_t s);
// Pass 2/3: w64 = w - V h (w read as TS when w64_in == null, else from w64_in);
// DOT: also partial dots of V^H w64; always pnrm = |w64|^2 partials.
template <typename TS>
void launch_update(const TS* V, int64_t ldv, int p, const double2* h, const TS* w_in,
                   const void* w64_in, void* w64_out, int64_t n, bool dot, double2* partial, double* pnrm,
                   hipStream_t s);
// beta = sqrt(sum pnrm); H[j+1, j] = beta; breakdown / non-finite flags.
void launch_finalize(const double* pnrm, int nblk, const double* scal, int win_slot, double2* Hsub,
                     double* beta_out, RitzResult* rr, hipStream_t s);
// v = w64 / beta (stored as TS).
template <typename TS>
void launch_scale(const void* w64, const double* beta, TS* v, int64_t n, hipStream_t s);
// v = x / ||x|| from a state vector x (norm from scal[slot]).
template <typename TS>
void launch_scale_state(const TS* x, const double* scal, int slot, TS* v, int64_t n, hipStream_t s);
// X[s*n + e] = sum_i V_i[e] Y[s*p + i] (Y: unit Ritz coordinates of the k
// wanted pairs, in wanted order), complex128 output.
template <typename TS>
void launch_ritz_vectors(const TS* V, int64_t ldv, int p, const double2* Y, const int* sel, int k,
                         double2* X, int64_t n, hipStream_t s);
// Check a vector for NaN/Inf: flag[0] |= 1.
template <typename TS>
void launch_check_finite(const TS* x, int64_t n, int* flag, hipStream_t s);

}  // namespace tsk
