// Linearized 2D Navier-Stokes (vorticity form) about a general base flow
// (U(x, y), V(x, y)), pseudo-spectral with the 2/3 rule, Lawson
// integrating-factor RK4 (Sec. 3, eq. "linearized Navier-Stokes equations",
// curl taken):
//     d omega/dt = -(U d_x omega + V d_y omega + u d_x Omega + v d_y Omega)
//                  + Re^-1 lap omega,   u = d_y psi, v = -d_x psi, -lap psi = omega.
//
// Pipeline of one RK4 stage (the state and the RK4 bookkeeping stay in packed
// spectral form, see tsk.h):
//   column kernel (one workgroup of four wavefronts per kept kx column):
//     forward y-transform of the previous stage's product spectrum Q[kx][y],
//     RHS on the kept modes, RK4 update, then the four derived spectral fields
//     i kx s, i ky s, i ky s/K^2, -i kx s/K^2 of the next stage input s, one
//     per wavefront, and their inverse y-transforms into G[f][kx][y];
//   row kernel (one workgroup of 2 R wavefronts per R = 2 grid rows):
//     the four fields of each row by two concurrent complex inverse
//     x-transforms (two Hermitian half-spectra packed as a + i b per
//     transform), the products P = U d_x w + V d_y w + u Omega_x + v Omega_y
//     with the base fields, and one complex forward x-transform per row pair
//     (P0 + i P1), unpacked to the kx = 0..M half spectra Q[kx][y].
// G and Q are the only fields in HBM between the two kernels: each kernel
// reads and writes them once per stage (4 + 1 complex N x (M+1) arrays) and
// the row kernel reads the four base fields.  Running the four inverse
// transforms of a workgroup concurrently keeps the dependent chain of each
// kernel at two transforms.  The x- and y-transforms are the Stockham LDS FFTs
// of fft.hpp.
//
// Scaling.  Packed coefficients c = sqrt(2) rfft2(omega)/N^2.  The derived
// fields are formed from c directly and the transforms are unnormalised, so
// the products are sqrt(2) times the physical ones; the RHS in packed units is
// then -rfft2(P')/N^2 with no further sqrt(2).
#include <cmath>
#include <vector>

#include "fft.hpp"
#include "kolmo2d.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

template <int N> struct Geo2 {
    static constexpr int M = (N - 1) / 3;
    static constexpr int MC = M + 1;     // kept kx columns
    static constexpr int NM = 2 * M + 1;  // kept ky per column (kx > 0)
    static __host__ __device__ constexpr int64_t seg(int kx) {
        return kx == 0 ? 0 : 2ll * M + int64_t(kx - 1) * 2 * NM;
    }
};

constexpr int kGT = 4 * kWave;  // column kernel: four wavefronts per workgroup

// Row groups of the row kernels by XCD.  The device has 8 XCDs, each with its
// own L2, and hands workgroups to them in turn (workgroup b runs on XCD b mod
// 8).  The row kernels read G and write Q with y the fastest index, so the
// rows of one 128-byte line (8 FP64 or 16 FP32 complex values) belong to
// several workgroups; numbered in launch order, those workgroups sit on
// different XCDs and each XCD's L2 fetches the whole line.  Workgroup b
// therefore takes row group (b mod 8) (nb / 8) + b / 8: each XCD gets a
// contiguous band of nb / 8 groups, and a line is fetched by one L2 only once
// the band covers it (nb / 8 >= 4 at two rows per group, N >= 64).
__device__ inline int xcd_row_group(int b, int nb) {
    constexpr int kXcd = 8;
    return nb % kXcd == 0 ? (b % kXcd) * (nb / kXcd) + b / kXcd : b;
}

enum GenMode { GEN_FIRST = 0, GEN_STAGE = 1, GEN_LAST = 2 };

// Column kernel, one workgroup per kept kx column.  FIRST: W = x, s = W,
// derived fields of s.  STAGE: RHS from Q, RK4 stage q, derived fields of the
// next stage input.  LAST: RHS from Q, final stage (q = 3), y = new W.  The
// forward transform and the RK4 update use the whole workgroup; wavefront f
// then forms derived field f and runs its inverse transform, the four
// concurrently.
template <typename real, int N>
__global__ __launch_bounds__(kGT) void k_gen_col(const real* __restrict__ xin, real* __restrict__ W,
                                                 real* __restrict__ Acc, const cplx<real>* __restrict__ Q,
                                                 cplx<real>* __restrict__ Gf, real* __restrict__ yout,
                                                 const cplx<real>* __restrict__ twg, double alpha, double Re,
                                                 double dt, int q, int mode, const real* __restrict__ fvec) {
    using C = cplx<real>;
    using G = Geo2<N>;
    constexpr int M = G::M, MC = G::MC, NM = G::NM;
    __shared__ C sA[4][N], sB[4][N], sT[N];
    __shared__ C sS[NM];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave, kx = blockIdx.x;
    const int nq = kx == 0 ? M : NM;  // packed complex entries of the column
    const int64_t base = G::seg(kx);
    for (int t = tid; t < N; t += kGT) sT[t] = twg[t];
    const double kxv = alpha * kx;

    if (mode == GEN_FIRST) {
        for (int e = tid; e < nq; e += kGT) {
            const real re = xin[base + 2 * e], im = xin[base + 2 * e + 1];
            W[base + 2 * e] = re;
            W[base + 2 * e + 1] = im;
            sS[e] = cmk<C>(re, im);
        }
        __syncthreads();
    } else {
        // the thread's modes e = tid + kGT r: W, Acc (and the forcing) are loaded
        // first, so their latency overlaps the load and transform of Q
        constexpr int R = (NM + kGT - 1) / kGT;
        real wv[R][2], av[R][2], fv[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + kGT * r;
            const int64_t o = base + 2 * (e < nq ? e : 0);
            wv[r][0] = W[o];
            wv[r][1] = W[o + 1];
            av[r][0] = q == 0 ? real(0) : Acc[o];
            av[r][1] = q == 0 ? real(0) : Acc[o + 1];
            fv[r][0] = fvec ? fvec[o] : real(0);
            fv[r][1] = fvec ? fvec[o + 1] : real(0);
        }
        for (int t = tid; t < N; t += kGT) sA[0][t] = Q[size_t(kx) * N + t];
        __syncthreads();
        const C* X = fft_lds<N, -1, kGT>(sA[0], sB[0], sT, tid);
        const double h = dt, h2 = 0.5 * dt, h3 = dt / 3.0, h6 = dt / 6.0;
        const double scl = -1.0 / (double(N) * N);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + kGT * r;
            if (e >= nq) continue;
            const int jy = kx == 0 ? e + 1 : e - M;
            const C xr = X[jy < 0 ? jy + N : jy];
            // steady forcing (packed units) of the nonlinear equation, else 0
            const double nx = scl * double(xr.x) + double(fv[r][0]), ny = scl * double(xr.y) + double(fv[r][1]);
            const double K2 = kxv * kxv + double(jy) * jy;
            const double e1 = exp(-K2 * dt / Re), eh = exp(-K2 * (0.5 * dt) / Re);
            const int64_t o = base + 2 * e;
            const double wx = wv[r][0], wy = wv[r][1];
            const double ax = av[r][0], ay = av[r][1];
            double sx, sy;
            if (q == 0) {
                Acc[o] = real(e1 * (wx + h6 * nx));
                Acc[o + 1] = real(e1 * (wy + h6 * ny));
                sx = eh * (wx + h2 * nx);
                sy = eh * (wy + h2 * ny);
            } else if (q == 1) {
                Acc[o] = real(ax + h3 * eh * nx);
                Acc[o + 1] = real(ay + h3 * eh * ny);
                sx = eh * wx + h2 * nx;
                sy = eh * wy + h2 * ny;
            } else if (q == 2) {
                Acc[o] = real(ax + h3 * eh * nx);
                Acc[o + 1] = real(ay + h3 * eh * ny);
                sx = e1 * wx + h * eh * nx;
                sy = e1 * wy + h * eh * ny;
            } else {
                const real nwx = real(ax + h6 * nx), nwy = real(ay + h6 * ny);
                if (mode == GEN_LAST) {
                    yout[o] = nwx;
                    yout[o + 1] = nwy;
                } else {
                    W[o] = nwx;
                    W[o + 1] = nwy;
                }
                sx = nwx;
                sy = nwy;
            }
            sS[e] = cmk<C>(real(sx), real(sy));
        }
        __syncthreads();
        if (mode == GEN_LAST) return;
    }
    // wavefront f: derived field f of s (i g s, g = kx, ky, ky/K^2, -kx/K^2) and
    // its inverse y-transform
    C* a = sA[wv];
    C* b = sB[wv];
    for (int t = lane; t < N; t += kWave) a[t] = cmk<C>(real(0), real(0));
    __syncthreads();
    for (int e = lane; e < nq; e += kWave) {
        const int jy = kx == 0 ? e + 1 : e - M;
        const double K2 = kxv * kxv + double(jy) * jy;
        const C sv = sS[e];
        const double g = wv == 0 ? kxv : wv == 1 ? double(jy) : wv == 2 ? double(jy) / K2 : -kxv / K2;
        const C d = cmk<C>(real(-g * double(sv.y)), real(g * double(sv.x)));
        a[jy < 0 ? jy + N : jy] = d;
        if (kx == 0) a[N - jy] = cconj(d);
    }
    __syncthreads();
    const C* X = fft_lds<N, +1, kWave>(a, b, sT, lane);
    C* out = Gf + (size_t(wv) * MC + kx) * N;
    for (int t = lane; t < N; t += kWave) out[t] = X[t];
}

// Row kernel, one workgroup per RPW consecutive grid rows y0 .. y0 + RPW - 1
// (gen_rows_per_group).  Wavefront 2r + pr
// inverse-transforms field pair pr ((d_x w, d_y w) or (u, v), packed as a + i b)
// of row y0 + r; the workgroup then forms the products of all its rows and
// transforms them forward two rows at a time (P_2a + i P_2a+1, 256 threads per
// transform, the RPW/2 transforms concurrently).
//   ROW_LIN:    P = U d_x w + V d_y w + u Omega_x + v Omega_y (base fields U..Oy);
//   ROW_NL:     P = (u + U0) d_x w + v d_y w of the state itself (nonlinear
//               advection; the derived fields carry the packing factor sqrt(2),
//               so their product is divided by sqrt(2) once);
//   ROW_FIELDS: no product: the physical grid fields (u + U0, v, d_x w, d_y w)
//               of the state go to U, V, Ox, Oy (the state as a base flow).
enum RowMode { ROW_LIN = 0, ROW_NL = 1, ROW_FIELDS = 2 };
// Rows per workgroup: 2 (whole 128-byte lines per L2 come from the row groups
// by XCD, xcd_row_group).  With 8 rows (16 wavefronts) one workgroup covers
// whole lines by itself, but its 16 workgroups of 1024 threads take 9.6
// instead of 5.4 us per launch at 128^2 (4 rows: 6.8 us); the stage is
// latency-bound, so the wider grid of small workgroups wins.
template <typename real, int N> constexpr int gen_rows_per_group() {
    return 2;
}
template <typename real, int N, int RM, int RPW>
__global__ __launch_bounds__(2 * RPW * kWave) void k_gen_row(const cplx<real>* __restrict__ Gf, real* __restrict__ U,
                                                             real* __restrict__ V, real* __restrict__ Ox,
                                                             real* __restrict__ Oy, cplx<real>* __restrict__ Q,
                                                             const cplx<real>* __restrict__ twg, double U0) {
    using C = cplx<real>;
    using G = Geo2<N>;
    constexpr int M = G::M, MC = G::MC;
    constexpr int NT = 2 * RPW * kWave;  // threads
    constexpr int NP = RPW / 2;          // row pairs, one forward transform each
    constexpr int GT = NT / NP;          // threads per forward transform
    constexpr int NE = RPW * N;          // grid points of the workgroup
    constexpr int RX = (NE + NT - 1) / NT;
    static_assert(N % RPW == 0 && GT == 4 * kWave, "row grouping");
    __shared__ C sT[N];
    __shared__ C sA[2 * RPW][N], sB[2 * RPW][N];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int y0 = RPW * xcd_row_group(blockIdx.x, gridDim.x), r = wv >> 1, pr = wv & 1, y = y0 + r;
    // the base fields of the thread's grid points (ROW_LIN), loaded first so that
    // their latency overlaps the transforms; point e = rr N + x of the workgroup
    real bU[RX], bV[RX], bOx[RX], bOy[RX];
    if constexpr (RM == ROW_LIN) {
#pragma unroll
        for (int i = 0; i < RX; ++i) {
            const int e = tid + NT * i;
            const size_t o = size_t(y0) * N + (e < NE ? e : 0);
            bU[i] = U[o];
            bV[i] = V[o];
            bOx[i] = Ox[o];
            bOy[i] = Oy[o];
        }
    }
    for (int t = tid; t < N; t += NT) sT[t] = twg[t];
    C* a = sA[wv];
    C* b = sB[wv];
    for (int t = lane; t < N; t += kWave) a[t] = cmk<C>(real(0), real(0));
    __syncthreads();
    const C* g1s = Gf + (size_t(2 * pr) * MC) * N + y;
    const C* g2s = Gf + (size_t(2 * pr + 1) * MC) * N + y;
    for (int k = lane; k <= M; k += kWave) {
        C g1 = g1s[size_t(k) * N], g2 = g2s[size_t(k) * N];
        if (k == 0) {  // the kx = 0 column of a real field is real
            g1.y = real(0);
            g2.y = real(0);
        }
        a[k] = cmk<C>(g1.x - g2.y, g1.y + g2.x);                 // g1 + i g2
        if (k > 0) a[N - k] = cmk<C>(g1.x + g2.y, g2.x - g1.y);  // conj(g1) + i conj(g2)
    }
    __syncthreads();
    fft_lds<N, +1, kWave>(a, b, sT, lane);
    __syncthreads();
    // the inverse results of row rr sit in sA[2 rr + pr] after an even number of
    // passes, else in sB; the other set is free for the products
    constexpr bool in_a = fft_num_passes(N) % 2 == 0;
    C(*res)[N] = in_a ? sA : sB;
    C(*freeb)[N] = in_a ? sB : sA;
    if constexpr (RM == ROW_FIELDS) {
        const real is2 = real(0.70710678118654752440);  // packing factor sqrt(2) removed
        for (int e = tid; e < NE; e += NT) {
            const int rr = e / N, x = e % N;
            const size_t o = size_t(y0) * N + e;
            const C d = res[2 * rr][x], uv = res[2 * rr + 1][x];
            U[o] = is2 * uv.x + real(U0);
            V[o] = is2 * uv.y;
            Ox[o] = is2 * d.x;
            Oy[o] = is2 * d.y;
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < RX; ++i) {
        const int e = tid + NT * i;
        if (e >= NE) continue;
        const int rr = e / N, x = e % N;
        const C d = res[2 * rr][x], uv = res[2 * rr + 1][x];  // (d_x w, d_y w), (u, v)
        real pv;
        if constexpr (RM == ROW_NL) {
            const real is2 = real(0.70710678118654752440), u0 = real(U0);
            pv = is2 * (uv.x * d.x + uv.y * d.y) + u0 * d.x;
        } else {
            pv = bU[i] * d.x + bV[i] * d.y + bOx[i] * uv.x + bOy[i] * uv.y;
        }
        C* z = freeb[2 * (rr >> 1)];
        if (rr & 1) z[x].y = pv;
        else z[x].x = pv;
    }
    __syncthreads();
    const int g = tid / GT, gt = tid % GT;  // transform g: rows 2g, 2g + 1
    const C* Z = fft_lds<N, -1, GT>(freeb[2 * g], freeb[2 * g + 1], sT, gt);
    for (int k = gt; k <= M; k += GT) {
        const C za = Z[k], zb = cconj(Z[k == 0 ? 0 : N - k]);
        Q[size_t(k) * N + y0 + 2 * g] = cmk<C>(real(0.5) * (za.x + zb.x), real(0.5) * (za.y + zb.y));
        Q[size_t(k) * N + y0 + 2 * g + 1] = cmk<C>(real(0.5) * (za.y - zb.y), real(-0.5) * (za.x - zb.x));
    }
}

// ---- the transposed pipeline (discrete adjoint) ------------------------------------
// The advection operator of a stage is N s = -R sum_f B_f P(D_f s): D_f the four
// derived fields i c_f s (c = kx, ky, ky/K^2, -kx/K^2), P packed state -> grid
// field, B_f the base fields (U, V, Omega_x, Omega_y), R grid field -> packed
// state on the kept modes.  The packed Euclidean norm is the RMS of the field,
// so P^T = N^2 R; D_f^T = -D_f; B_f is symmetric.  Hence
//     N^T v = sum_f D_f R(B_f P v) = (1/N^2) sum_f i c_f F(B_f F^-1 v)
// with the pipeline's unnormalised transforms (the sqrt(2) of the packing
// cancels): one inverse 2-D transform of v, four products, four forward
// transforms.  The Lawson step transposes stage by stage in reverse order, as
// for the column steppers (z the adjoint state, so the stage output):
//     so3 = N^T(h/6 z),                acc = E1 z + E1 so3
//     so2 = N^T(h/3 Eh z + h Eh so3),  acc += Eh so2
//     so1 = N^T(h/3 Eh z + h/2 so2),   acc += Eh so1
//     so0 = N^T(h/6 E1 z + h/2 Eh so1), z+ = acc + so0.
// A stage is one row kernel (the inverse x-transform of two rows of v packed as
// a + i b, the products, four forward x-transforms) and one column kernel (four
// forward y-transforms, the stage output and the RK bookkeeping, the next
// stage input and its inverse y-transform).  The exchanged arrays swap roles:
// G1 [kx][y] (one field, the Q buffer) and Q4 [f][kx][y] (four, the G buffer).

// Column kernel of the transposed pipeline, one workgroup per kept kx column.
// FIRST: z = x, next input h/6 z.  STAGE q: so from Q4, RK bookkeeping of stage
// q (W holds z, Acc acc), the next stage input.  LAST (stage 3 of the last
// step): y = new z.
template <typename real, int N>
__global__ __launch_bounds__(kGT) void k_gen_col_adj(const real* __restrict__ xin, real* __restrict__ W,
                                                     real* __restrict__ Acc, const cplx<real>* __restrict__ Q4,
                                                     cplx<real>* __restrict__ G1, real* __restrict__ yout,
                                                     const cplx<real>* __restrict__ twg, double alpha, double Re,
                                                     double dt, int q, int mode) {
    using C = cplx<real>;
    using G = Geo2<N>;
    constexpr int M = G::M, MC = G::MC, NM = G::NM;
    __shared__ C sA[4][N], sB[4][N], sT[N];
    __shared__ C sS[NM];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave, kx = blockIdx.x;
    const int nq = kx == 0 ? M : NM;  // packed complex entries of the column
    const int64_t base = G::seg(kx);
    for (int t = tid; t < N; t += kGT) sT[t] = twg[t];
    const double kxv = alpha * kx;
    const double h = dt, h2 = 0.5 * dt, h3 = dt / 3.0, h6 = dt / 6.0;

    if (mode == GEN_FIRST) {
        for (int e = tid; e < nq; e += kGT) {
            const real re = xin[base + 2 * e], im = xin[base + 2 * e + 1];
            W[base + 2 * e] = re;
            W[base + 2 * e + 1] = im;
            sS[e] = cmk<C>(real(h6 * double(re)), real(h6 * double(im)));
        }
        __syncthreads();
    } else {
        constexpr int R = (NM + kGT - 1) / kGT;
        real zv[R][2], av[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + kGT * r;
            const int64_t o = base + 2 * (e < nq ? e : 0);
            zv[r][0] = W[o];
            zv[r][1] = W[o + 1];
            av[r][0] = q == 0 ? real(0) : Acc[o];
            av[r][1] = q == 0 ? real(0) : Acc[o + 1];
        }
        // wavefront f: forward y-transform of field f's column
        for (int t = lane; t < N; t += kWave) sA[wv][t] = Q4[(size_t(wv) * MC + kx) * N + t];
        __syncthreads();
        fft_lds<N, -1, kWave>(sA[wv], sB[wv], sT, lane);
        __syncthreads();
        constexpr bool in_a = fft_num_passes(N) % 2 == 0;
        const double scl = 1.0 / (double(N) * N);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + kGT * r;
            if (e >= nq) continue;
            const int jy = kx == 0 ? e + 1 : e - M;
            const int ix = jy < 0 ? jy + N : jy;
            const double K2 = kxv * kxv + double(jy) * jy;
            const double cf[4] = {kxv, double(jy), double(jy) / K2, -kxv / K2};
            double sx = 0.0, sy = 0.0;  // so = (1/N^2) sum_f i c_f X_f
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const C xf = in_a ? sA[f][ix] : sB[f][ix];
                sx -= cf[f] * double(xf.y);
                sy += cf[f] * double(xf.x);
            }
            sx *= scl;
            sy *= scl;
            const double e1 = exp(-K2 * dt / Re), eh = exp(-K2 * (0.5 * dt) / Re);
            const int64_t o = base + 2 * e;
            const double zx = zv[r][0], zy = zv[r][1];
            double vx, vy;  // the next stage's input
            if (q == 0) {
                Acc[o] = real(e1 * (zx + sx));
                Acc[o + 1] = real(e1 * (zy + sy));
                vx = eh * (h3 * zx + h * sx);
                vy = eh * (h3 * zy + h * sy);
            } else if (q == 1) {
                Acc[o] = real(double(av[r][0]) + eh * sx);
                Acc[o + 1] = real(double(av[r][1]) + eh * sy);
                vx = h3 * eh * zx + h2 * sx;
                vy = h3 * eh * zy + h2 * sy;
            } else if (q == 2) {
                Acc[o] = real(double(av[r][0]) + eh * sx);
                Acc[o + 1] = real(double(av[r][1]) + eh * sy);
                vx = h6 * e1 * zx + h2 * eh * sx;
                vy = h6 * e1 * zy + h2 * eh * sy;
            } else {
                const real nzx = real(double(av[r][0]) + sx), nzy = real(double(av[r][1]) + sy);
                if (mode == GEN_LAST) {
                    yout[o] = nzx;
                    yout[o + 1] = nzy;
                } else {
                    W[o] = nzx;
                    W[o + 1] = nzy;
                }
                vx = h6 * double(nzx);
                vy = h6 * double(nzy);
            }
            sS[e] = cmk<C>(real(vx), real(vy));
        }
        __syncthreads();
        if (mode == GEN_LAST) return;
    }
    // the next stage input v of the column and its inverse y-transform (all four wavefronts)
    C* a = sA[0];
    for (int t = tid; t < N; t += kGT) a[t] = cmk<C>(real(0), real(0));
    __syncthreads();
    for (int e = tid; e < nq; e += kGT) {
        const int jy = kx == 0 ? e + 1 : e - M;
        const C v = sS[e];
        a[jy < 0 ? jy + N : jy] = v;
        if (kx == 0) a[N - jy] = cconj(v);  // the kx = 0 column of a real field
    }
    __syncthreads();
    const C* X = fft_lds<N, +1, kGT>(a, sB[0], sT, tid);
    C* out = G1 + size_t(kx) * N;
    for (int t = tid; t < N; t += kGT) out[t] = X[t];
}

// Row kernel of the transposed pipeline, one workgroup per pair of grid rows
// (y0, y0 + 1): the inverse x-transform of both rows of v (packed as a + i b),
// the four products with the base fields, and wavefront f's forward
// x-transform of field f of both rows (P_f,0 + i P_f,1), unpacked to the
// kx = 0..M half spectra Q4[f][kx][y].
template <typename real, int N>
__global__ __launch_bounds__(kGT) void k_gen_row_adj(const cplx<real>* __restrict__ G1, const real* __restrict__ U,
                                                     const real* __restrict__ V, const real* __restrict__ Ox,
                                                     const real* __restrict__ Oy, cplx<real>* __restrict__ Q4,
                                                     const cplx<real>* __restrict__ twg) {
    using C = cplx<real>;
    using G = Geo2<N>;
    constexpr int M = G::M, MC = G::MC;
    constexpr int RX = (N + kGT - 1) / kGT;
    __shared__ C sT[N];
    __shared__ C sA[4][N], sB[4][N];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int y0 = 2 * xcd_row_group(blockIdx.x, gridDim.x);
    // base fields of the thread's points of both rows, loaded first
    real bf[RX][4][2];
#pragma unroll
    for (int r = 0; r < RX; ++r) {
        const int x = tid + kGT * r < N ? tid + kGT * r : 0;
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const size_t o = size_t(y0 + rr) * N + x;
            bf[r][0][rr] = U[o];
            bf[r][1][rr] = V[o];
            bf[r][2][rr] = Ox[o];
            bf[r][3][rr] = Oy[o];
        }
    }
    for (int t = tid; t < N; t += kGT) sT[t] = twg[t];
    C* a = sA[0];
    for (int t = tid; t < N; t += kGT) a[t] = cmk<C>(real(0), real(0));
    __syncthreads();
    for (int k = tid; k <= M; k += kGT) {
        C g0 = G1[size_t(k) * N + y0], g1 = G1[size_t(k) * N + y0 + 1];
        if (k == 0) {  // the kx = 0 column of a real field is real
            g0.y = real(0);
            g1.y = real(0);
        }
        a[k] = cmk<C>(g0.x - g1.y, g0.y + g1.x);                 // g0 + i g1
        if (k > 0) a[N - k] = cmk<C>(g0.x + g1.y, g1.x - g0.y);  // conj(g0) + i conj(g1)
    }
    __syncthreads();
    const C* Fv = fft_lds<N, +1, kGT>(a, sB[0], sT, tid);  // v of row y0 + i v of row y0 + 1
    // the products of field f go to a buffer not holding Fv: sA[1..3] and sB[1..3]
    // are free, and the fourth is whichever of sA[0] / sB[0] Fv is not in
    C* zf[4];
    C* sc[4];
    zf[0] = (Fv == sA[0]) ? sB[0] : sA[0];
    sc[0] = sA[1];
    zf[1] = sB[1];
    sc[1] = sA[2];
    zf[2] = sB[2];
    sc[2] = sA[3];
    zf[3] = sB[3];
    __shared__ C sExtra[N];
    sc[3] = sExtra;
#pragma unroll
    for (int r = 0; r < RX; ++r) {
        const int x = tid + kGT * r;
        if (x >= N) continue;
        const C v = Fv[x];
#pragma unroll
        for (int f = 0; f < 4; ++f) zf[f][x] = cmk<C>(bf[r][f][0] * v.x, bf[r][f][1] * v.y);
    }
    __syncthreads();
    const C* Z = fft_lds<N, -1, kWave>(zf[wv], sc[wv], sT, lane);
    C* Qf = Q4 + size_t(wv) * MC * N;
    for (int k = lane; k <= M; k += kWave) {
        const C za = Z[k], zb = cconj(Z[k == 0 ? 0 : N - k]);
        Qf[size_t(k) * N + y0] = cmk<C>(real(0.5) * (za.x + zb.x), real(0.5) * (za.y + zb.y));
        Qf[size_t(k) * N + y0 + 1] = cmk<C>(real(0.5) * (za.y - zb.y), real(-0.5) * (za.x - zb.x));
    }
}

// nsteps transposed Lawson steps from x into y (G1 in the Q buffer, Q4 in G).
template <typename real, int N>
void gen_run_adj(const void* x, void* y, real* W, real* Acc, cplx<real>* G1, cplx<real>* Q4, const real* U,
                 const real* V, const real* Ox, const real* Oy, const void* tw, double alpha, double Re, double dt,
                 int nsteps, hipStream_t s) {
    using C = cplx<real>;
    constexpr int MC = Geo2<N>::MC;
    const C* twc = static_cast<const C*>(tw);
    hipLaunchKernelGGL((k_gen_col_adj<real, N>), dim3(MC), dim3(kGT), 0, s, static_cast<const real*>(x), W, Acc, Q4,
                       G1, static_cast<real*>(y), twc, alpha, Re, dt, 0, int(GEN_FIRST));
    for (int st = 0; st < nsteps; ++st)
        for (int q = 0; q < 4; ++q) {
            hipLaunchKernelGGL((k_gen_row_adj<real, N>), dim3(N / 2), dim3(kGT), 0, s, G1, U, V, Ox, Oy, Q4, twc);
            const int mode = (st == nsteps - 1 && q == 3) ? GEN_LAST : GEN_STAGE;
            hipLaunchKernelGGL((k_gen_col_adj<real, N>), dim3(MC), dim3(kGT), 0, s, static_cast<const real*>(x), W,
                               Acc, Q4, G1, static_cast<real*>(y), twc, alpha, Re, dt, q, mode);
        }
}

template <typename real>
void gen_dispatch_adj(int N, const void* x, void* y, real* W, real* Acc, cplx<real>* G1, cplx<real>* Q4,
                      const real* U, const real* V, const real* Ox, const real* Oy, const void* tw, double alpha,
                      double Re, double dt, int nsteps, hipStream_t s) {
    switch (N) {
#define X(n)                                                                                                      \
    case n:                                                                                                       \
        gen_run_adj<real, n>(x, y, W, Acc, G1, Q4, U, V, Ox, Oy, tw, alpha, Re, dt, nsteps, s);                   \
        break;
        X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#undef X
    }
}

// One run of the pipeline.  ROW_LIN / ROW_NL: nsteps Lawson steps of the
// linearized / nonlinear (forcing fvec, drift U0) equation from x into y.
// ROW_FIELDS: the grid fields of x into U, V, Ox, Oy (nsteps ignored).
template <typename real, int N, int RM>
void gen_run(const void* x, void* y, real* W, real* Acc, cplx<real>* Q, cplx<real>* Gf, real* U, real* V, real* Ox,
             real* Oy, const void* tw, double alpha, double Re, double dt, int nsteps, double U0, const real* fvec,
             hipStream_t s) {
    using C = cplx<real>;
    constexpr int MC = Geo2<N>::MC;
    constexpr int RPW = gen_rows_per_group<real, N>();
    const C* twc = static_cast<const C*>(tw);
    hipLaunchKernelGGL((k_gen_col<real, N>), dim3(MC), dim3(kGT), 0, s, static_cast<const real*>(x), W, Acc, Q, Gf,
                       static_cast<real*>(y), twc, alpha, Re, dt, 0, int(GEN_FIRST), fvec);
    if constexpr (RM == ROW_FIELDS) {
        hipLaunchKernelGGL((k_gen_row<real, N, RM, RPW>), dim3(N / RPW), dim3(2 * RPW * kWave), 0, s, Gf, U, V, Ox,
                           Oy, Q, twc, U0);
        return;
    }
    for (int st = 0; st < nsteps; ++st)
        for (int q = 0; q < 4; ++q) {
            hipLaunchKernelGGL((k_gen_row<real, N, RM, RPW>), dim3(N / RPW), dim3(2 * RPW * kWave), 0, s, Gf, U, V,
                               Ox, Oy, Q, twc, U0);
            const int mode = (st == nsteps - 1 && q == 3) ? GEN_LAST : GEN_STAGE;
            hipLaunchKernelGGL((k_gen_col<real, N>), dim3(MC), dim3(kGT), 0, s, static_cast<const real*>(x), W, Acc,
                               Q, Gf, static_cast<real*>(y), twc, alpha, Re, dt, q, mode, fvec);
        }
}

template <typename real, int RM>
void gen_dispatch(int N, const void* x, void* y, real* W, real* Acc, cplx<real>* Q, cplx<real>* Gf, real* U, real* V,
                  real* Ox, real* Oy, const void* tw, double alpha, double Re, double dt, int nsteps, double U0,
                  const real* fvec, hipStream_t s) {
    switch (N) {
#define X(n)                                                                                                      \
    case n:                                                                                                       \
        gen_run<real, n, RM>(x, y, W, Acc, Q, Gf, U, V, Ox, Oy, tw, alpha, Re, dt, nsteps, U0, fvec, s);          \
        break;
        X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#undef X
    }
}

}  // namespace

struct Gen2D {
    int N = 0, M = 0;
    bool fp32 = false;
    DevBuf U, V, Ox, Oy, W, Acc, Q, G;
};

tsk_status gen2d_create(int N, bool fp32, const double* U, const double* V, const double* Ox, const double* Oy,
                        Gen2D** out) {
    auto g = std::make_unique<Gen2D>();
    g->N = N;
    g->M = (N - 1) / 3;
    g->fp32 = fp32;
    const size_t rb = fp32 ? 4 : 8, nn = size_t(N) * N;
    const int64_t n = 4ll * g->M * (g->M + 1);
    const double* src[4] = {U, V, Ox, Oy};
    DevBuf* dst[4] = {&g->U, &g->V, &g->Ox, &g->Oy};
    for (int f = 0; f < 4; ++f) {
        TSK_TRY(dst[f]->ensure(nn * rb));
        if (!src[f]) continue;  // filled on the device (gen2d_fields)
        if (fp32) {
            std::vector<float> h(src[f], src[f] + nn);
            TSK_HIP(hipMemcpy(dst[f]->ptr, h.data(), nn * 4, hipMemcpyHostToDevice));
        } else {
            TSK_HIP(hipMemcpy(dst[f]->ptr, src[f], nn * 8, hipMemcpyHostToDevice));
        }
    }
    TSK_TRY(g->W.ensure(size_t(n) * rb));
    TSK_TRY(g->Acc.ensure(size_t(n) * rb));
    TSK_TRY(g->Q.ensure(size_t(g->M + 1) * N * 2 * rb));
    TSK_TRY(g->G.ensure(4 * size_t(g->M + 1) * N * 2 * rb));
    *out = g.release();
    return TSK_OK;
}

void gen2d_free(Gen2D* g) { delete g; }

namespace {
template <int RM>
tsk_status gen_go(Gen2D* g, double alpha, double Re, double dt, int nsteps, double U0, const void* fvec, const void* x,
                  void* y, const void* tw, hipStream_t s) {
    if (g->fp32)
        gen_dispatch<float, RM>(g->N, x, y, g->W.as<float>(), g->Acc.as<float>(), g->Q.as<float2>(),
                                g->G.as<float2>(), g->U.as<float>(), g->V.as<float>(), g->Ox.as<float>(),
                                g->Oy.as<float>(), tw, alpha, Re, dt, nsteps, U0, static_cast<const float*>(fvec), s);
    else
        gen_dispatch<double, RM>(g->N, x, y, g->W.as<double>(), g->Acc.as<double>(), g->Q.as<double2>(),
                                 g->G.as<double2>(), g->U.as<double>(), g->V.as<double>(), g->Ox.as<double>(),
                                 g->Oy.as<double>(), tw, alpha, Re, dt, nsteps, U0, static_cast<const double*>(fvec),
                                 s);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}
}  // namespace

tsk_status gen2d_apply(Gen2D* g, double alpha, double Re, double dt, int nsteps, const void* x, void* y,
                       const void* tw, hipStream_t s) {
    return gen_go<ROW_LIN>(g, alpha, Re, dt, nsteps, 0.0, nullptr, x, y, tw, s);
}

tsk_status gen2d_apply_adjoint(Gen2D* g, double alpha, double Re, double dt, int nsteps, const void* x, void* y,
                               const void* tw, hipStream_t s) {
    if (g->fp32)
        gen_dispatch_adj<float>(g->N, x, y, g->W.as<float>(), g->Acc.as<float>(), g->Q.as<float2>(),
                                g->G.as<float2>(), g->U.as<float>(), g->V.as<float>(), g->Ox.as<float>(),
                                g->Oy.as<float>(), tw, alpha, Re, dt, nsteps, s);
    else
        gen_dispatch_adj<double>(g->N, x, y, g->W.as<double>(), g->Acc.as<double>(), g->Q.as<double2>(),
                                 g->G.as<double2>(), g->U.as<double>(), g->V.as<double>(), g->Ox.as<double>(),
                                 g->Oy.as<double>(), tw, alpha, Re, dt, nsteps, s);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status gen2d_nonlinear(Gen2D* g, double alpha, double Re, double dt, int nsteps, double U0, const void* fvec,
                           const void* x, void* y, const void* tw, hipStream_t s) {
    return gen_go<ROW_NL>(g, alpha, Re, dt, nsteps, U0, fvec, x, y, tw, s);
}

tsk_status gen2d_fields(Gen2D* g, double alpha, double U0, const void* x, const void* tw, hipStream_t s) {
    return gen_go<ROW_FIELDS>(g, alpha, 1.0, 1.0, 0, U0, nullptr, x, nullptr, tw, s);
}

}  // namespace tsk
