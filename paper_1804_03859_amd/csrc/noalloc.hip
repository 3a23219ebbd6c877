// Non-allocating variant of the standalone real Hessenberg eigensolver
// (tsk_hessenberg_ritz_real_noalloc), for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc.
//
// tsk_hessenberg_ritz_real allocates its scratch per call (a complex copy of H,
// the eigenvector workspace, the result record, device scalars and the
// descriptor the solver kernel reads).  This variant keeps the same scratch in
// one file-scope device array of fixed size, `scratch` below.  Every GPU the
// library runs on holds its own copy of it until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in
// symbol, not a device address): the address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that pointer is what the
// kernels get.  Every call on one device shares that device's array, so calls
// that overlap on one GPU (two host threads, or two streams) race; the last
// call's contents stay in it.  Everything the solver needs to start from zero
// (the result record, the scalars, the unused part of the complex copy) is
// rewritten by a fill kernel at the start of every call.
#include <cstring>
#include <mutex>

#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

// Largest order and leading dimension the scratch holds: the Arnoldi Hessenberg
// matrix of m <= 96 steps, (m + 1) x m with ldh = m + 1.
constexpr int kNoAllocMaxP = kMaxKrylov;
constexpr int kNoAllocMaxLdh = kMaxKrylov + 1;

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffDesc = 0;
constexpr size_t kOffRr = kOffDesc + align256(sizeof(KryDesc));
constexpr size_t kOffScal = kOffRr + align256(sizeof(RitzResult));
constexpr size_t kOffHc = kOffScal + align256(64 * sizeof(double));
constexpr size_t kOffS = kOffHc + align256(size_t(kNoAllocMaxLdh) * kNoAllocMaxP * sizeof(double2));
constexpr size_t kScratchBytes = kOffS + align256(size_t(kNoAllocMaxP) * kNoAllocMaxP * sizeof(double2));
static_assert(kScratchBytes < 320 * 1024, "the non-allocating scratch stays below 320 KB");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on the current device, looked up on the first call
// there and kept for the process.
tsk_status scratch_on_current_device(unsigned char** out) {
    static std::mutex mu;
    static unsigned char* ptr[64] = {};
    int dev = 0;
    TSK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(TSK_EINVAL, "device index beyond 63");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        TSK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(TSK_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
        ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = ptr[dev];
    return TSK_OK;
}

// Fill the scratch for one solve: the descriptor, a cleared result record, the
// scalars (beta in scal[2]) and the complex copy of H (real parts, zero
// imaginary parts) over all ldh x p entries the solver may read.
__global__ void k_noalloc_prep(const double* __restrict__ H, int ldh, int p, double beta, KryDesc d,
                               unsigned char* __restrict__ base) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double2* Hc = reinterpret_cast<double2*>(base + kOffHc);
    const int ne = ldh * p;
    for (int e = t; e < ne; e += gridDim.x * blockDim.x) Hc[e] = make_double2(H[e], 0.0);
    if (blockIdx.x == 0) {
        double* sc = reinterpret_cast<double*>(base + kOffScal);
        if (threadIdx.x < 64) sc[threadIdx.x] = threadIdx.x == 2 ? beta : 0.0;
        if (threadIdx.x == 0) {
            *reinterpret_cast<RitzResult*>(base + kOffRr) = RitzResult{};
            *reinterpret_cast<KryDesc*>(base + kOffDesc) = d;
        }
    }
}

}  // namespace

tsk_status hessenberg_ritz_real_noalloc(const double* H_dev, int ldh, int p, double beta, void* mu_dev,
                                        void* res_dev, hipStream_t s) {
    if (!H_dev || !mu_dev || !res_dev) return fail(TSK_EINVAL, "null buffer");
    if (p < 1 || p > kNoAllocMaxP)
        return fail(TSK_EINVAL, "p = " + std::to_string(p) + " is outside [1, 96], the largest order the "
                                "non-allocating scratch holds");
    if (ldh < p || ldh > kNoAllocMaxLdh)
        return fail(TSK_EINVAL, "ldh = " + std::to_string(ldh) + " must be in [p, 97] for the non-allocating "
                                "scratch");
    unsigned char* base = nullptr;
    TSK_TRY(scratch_on_current_device(&base));
    KryDesc d;
    std::memset(&d, 0, sizeof(d));
    d.H = reinterpret_cast<double2*>(base + kOffHc);
    d.ldh = ldh;
    d.scal = reinterpret_cast<double*>(base + kOffScal);
    d.S = reinterpret_cast<double2*>(base + kOffS);
    d.mu = static_cast<double2*>(mu_dev);
    d.res = static_cast<double*>(res_dev);
    d.rr = reinterpret_cast<RitzResult*>(base + kOffRr);
    d.active = 1;
    const int ne = ldh * p;
    const int blocks = (ne + 255) / 256;
    hipLaunchKernelGGL(k_noalloc_prep, dim3(blocks), dim3(256), 0, s, H_dev, ldh, p, beta, d, base);
    TSK_HIP(hipGetLastError());
    TSK_TRY(hess_ritz_launch(reinterpret_cast<const KryDesc*>(base + kOffDesc), 1, p, 0, 0.0, true, s, true));
    RitzResult h{};
    TSK_HIP(hipMemcpyAsync(&h, base + kOffRr, sizeof(RitzResult), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    if (h.nonfinite) return fail(TSK_ENONFINITE, "H or beta is not finite");
    if (h.eig_fail) return fail(TSK_EEIG, "Hessenberg QR did not converge");
    return TSK_OK;
}

}  // namespace tsk
