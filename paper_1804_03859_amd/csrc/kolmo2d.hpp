// Linearized Navier-Stokes about a general two-dimensional base flow: the full
// pseudo-spectral pipeline with two-dimensional transforms (kolmo2d.hip).
#pragma once

#include "common.hpp"

namespace tsk {

struct Gen2D;
// Base fields: N*N samples each ([y][x], FP64 on the host) of U, V, dOmega/dx and
// dOmega/dy, stored on the device in the operator's precision (null pointers:
// allocated only, to be filled by gen2d_fields).
tsk_status gen2d_create(int N, bool fp32, const double* U, const double* V, const double* Ox, const double* Oy,
                        Gen2D** out);
void gen2d_free(Gen2D* g);
// One matvec (T/dt = nsteps Lawson RK4 steps) of the packed state x into y.
// tw: exp(-2 pi i t / N), t < N, in the operator's precision (complex).
tsk_status gen2d_apply(Gen2D* g, double alpha, double Re, double dt, int nsteps, const void* x, void* y,
                       const void* tw, hipStream_t s);
// The transposed propagator (discrete adjoint in the packed Euclidean inner
// product) applied to x into y: nsteps transposed Lawson steps.
tsk_status gen2d_apply_adjoint(Gen2D* g, double alpha, double Re, double dt, int nsteps, const void* x, void* y,
                               const void* tw, hipStream_t s);
// nsteps Lawson steps of the nonlinear forced equation (advection (u + U0) d_x w +
// v d_y w of the state, steady forcing fvec in packed units) from x into y.
// The base-field arrays are not read.
tsk_status gen2d_nonlinear(Gen2D* g, double alpha, double Re, double dt, int nsteps, double U0, const void* fvec,
                           const void* x, void* y, const void* tw, hipStream_t s);
// The grid fields (u + U0, v, d_x w, d_y w) of the packed state x into g's base
// arrays (U, V, Omega_x, Omega_y): the state becomes the base flow of g.
tsk_status gen2d_fields(Gen2D* g, double alpha, double U0, const void* x, const void* tw, hipStream_t s);

}  // namespace tsk
