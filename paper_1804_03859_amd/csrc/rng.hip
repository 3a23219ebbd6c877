// Seeded N(0,1) draws for start vectors.
//
// Generator: splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014), used counter-style: output i of the
// sequence seeded with x0 is mix(x0 + (i+1) * 0x9e3779b97f4a7c15), so every
// element is computed independently.  Two consecutive outputs give two uniform
// doubles u = (o >> 11) 2^-53 in [0, 1), turned into two normal draws by the
// Box-Muller transform (Box & Muller 1958): r = sqrt(-2 ln(1 - u1)),
// z0 = r cos(2 pi u2), z1 = r sin(2 pi u2).  Element e takes z0 of pair e/2 if
// e is even, z1 otherwise.
#include "ops.hpp"

namespace tsk {

namespace {

__global__ void k_normal(double* __restrict__ out, int64_t count, uint64_t seed) {
    const int64_t npair = (count + 1) / 2;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < npair; q += int64_t(gridDim.x) * blockDim.x) {
        uint64_t o1 = splitmix_at(seed, 2 * uint64_t(q));
        uint64_t o2 = splitmix_at(seed, 2 * uint64_t(q) + 1);
        double u1 = double(o1 >> 11) * 0x1.0p-53;
        double u2 = double(o2 >> 11) * 0x1.0p-53;
        double r = sqrt(-2.0 * log(1.0 - u1));
        double th = 6.283185307179586476925286766559 * u2;
        double sn, cs;
        sincos(th, &sn, &cs);
        out[2 * q] = r * cs;
        if (2 * q + 1 < count) out[2 * q + 1] = r * sn;
    }
}

__global__ void k_narrow(const double* __restrict__ in, float* out, int64_t count) {
    // One thread per element, in index order within a block; a grid-stride loop
    // would let a later block overwrite doubles an earlier one has not read when
    // out aliases in, so the narrowing runs in a single block, sequentially in
    // chunks of blockDim values.
    for (int64_t base = 0; base < count; base += blockDim.x) {
        int64_t g = base + threadIdx.x;
        double v = g < count ? in[g] : 0.0;
        __syncthreads();
        if (g < count) out[g] = float(v);
        __syncthreads();
    }
}

}  // namespace

tsk_status normal_fill(double* out, int64_t count, uint64_t seed, hipStream_t s) {
    if (count <= 0) return TSK_OK;
    int64_t npair = (count + 1) / 2;
    int grid = int((npair + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_normal, dim3(grid), dim3(256), 0, s, out, count, seed);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

tsk_status narrow_to_float(const double* in, float* out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(k_narrow, dim3(1), dim3(1024), 0, s, in, out, count);
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

}  // namespace tsk
