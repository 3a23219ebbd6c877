// Linearized Navier-Stokes about a general two-dimensional base flow: the full
// pseudo-spectral pipeline with two-dimensional transforms (kolmo2d.hip).
#pragma once

#include "common.hpp"

namespace tsk {

struct Gen2D;
// Base fields: N*N samples each ([y][x], FP64 on the host) of U, V, dOmega/dx and
// dOmega/dy, stored on the device in the operator's precision.
tsk_status gen2d_create(int N, bool fp32, const double* U, const double* V, const double* Ox, const double* Oy,
                        Gen2D** out);
void gen2d_free(Gen2D* g);
// One matvec (T/dt = nsteps Lawson RK4 steps) of the packed state x into y.
// tw: exp(-2 pi i t / N), t < N, in the operator's precision (complex).
tsk_status gen2d_apply(Gen2D* g, double alpha, double Re, double dt, int nsteps, const void* x, void* y,
                       const void* tw, hipStream_t s);

}  // namespace tsk
