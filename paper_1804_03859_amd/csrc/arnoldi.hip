// Arnoldi driver (host orchestration of device kernels).
//
// m-step Arnoldi factorisation M V_m = V_m H_m + beta v_{m+1} e_m^T
// (Sec. 3.2.1, eq. "m-step Arnoldi", Algorithm 1) with every matvec a time
// integration of the linearized equations (Sec. 3, time-stepper approach).
// After each matvec: CGS2 projection and normalisation (krylov.hip), then the
// device Hessenberg QR and wanted-set test (hessenberg.hip).  The only device to
// host traffic per step is the 48-byte RitzResult that tells the host whether
// to stop.
//
// Overlap: as soon as v_{j+1} exists, the matvec M v_{j+1} is launched on the
// operator's stream while the Ritz analysis of H_j runs on a side stream (one
// wavefront, so it barely competes for compute units).  The host waits only for
// the side stream; if H_j already satisfies the stop test, the speculative
// matvec is discarded (it is neither counted nor used).  Ritz values are mapped to lambda = log(mu)/T on the device
// (principal branch, valid when |Im lambda| T < pi/2, the four-samples-per-period
// rule of Sec. 3.2.1).
#include <chrono>
#include <cstring>

#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

__global__ void k_gather_ritz(const double2* __restrict__ mu, const double* __restrict__ res,
                              const int* __restrict__ sel, int nsel, double T, double* __restrict__ out) {
    // out layout: [mu re,im]*nsel | [lambda re,im]*nsel | [res]*nsel
    int s = threadIdx.x;
    if (s >= nsel) return;
    double2 m = mu[sel[s]];
    out[2 * s] = m.x;
    out[2 * s + 1] = m.y;
    double r = hypot(m.x, m.y);
    out[2 * nsel + 2 * s] = log(r) / T;
    out[2 * nsel + 2 * s + 1] = atan2(m.y, m.x) / T;
    out[4 * nsel + s] = res[sel[s]];
}

template <typename TS> struct WorkType { using A = double; };
template <> struct WorkType<double2> { using A = double2; };

template <typename TS>
tsk_status arnoldi_t(Operator* op, int m, int k, double tol, const void* v0, uint64_t seed, double* mu_ri,
                     double* lam_ri, double* resid, void* ritz, tsk_arnoldi_info* info) {
    using A = typename WorkType<TS>::A;
    auto t0 = std::chrono::steady_clock::now();
    const hipStream_t s = op->stream;
    ArnoldiWork& W = op->aw;
    const int64_t n = op->n;
    const int64_t ldv = (n + 63) / 64 * 64;
    const int nblk = cgs_blocks(n);

    TSK_TRY(W.V.ensure(size_t(m + 1) * ldv * sizeof(TS)));
    TSK_TRY(W.H.ensure(size_t(m + 1) * m * sizeof(double2)));
    TSK_TRY(W.w.ensure(size_t(n) * sizeof(TS)));
    TSK_TRY(W.w64.ensure(size_t(n) * sizeof(A)));
    TSK_TRY(W.partial.ensure(size_t(nblk) * (m + 1) * sizeof(double2)));
    TSK_TRY(W.pnrm.ensure(size_t(nblk) * sizeof(double)));
    TSK_TRY(W.h.ensure(size_t(m + 1) * sizeof(double2)));
    TSK_TRY(W.scal.ensure(64 * sizeof(double)));
    TSK_TRY(W.eigZ.ensure(size_t(m) * m * sizeof(double2)));
    TSK_TRY(W.eigS.ensure(size_t(m) * m * sizeof(double2)));
    TSK_TRY(W.eigY.ensure(size_t(m) * m * sizeof(double2)));
    TSK_TRY(W.eigMu.ensure(size_t(m) * sizeof(double2)));
    TSK_TRY(W.eigRes.ensure(size_t(m) * sizeof(double)));
    const size_t gath_off = (size_t(m) * sizeof(int) + 15) / 16 * 16;
    TSK_TRY(W.sel.ensure(gath_off + 5 * size_t(k) * sizeof(double)));
    TSK_TRY(W.rr.ensure(sizeof(RitzResult)));
    if (!W.rr_host) TSK_HIP(hipHostMalloc((void**)&W.rr_host, sizeof(RitzResult) + 64 * sizeof(double), 0));
    while (W.ev_apply.size() < size_t(2 * (m + 1))) {
        hipEvent_t e;
        TSK_HIP(hipEventCreate(&e));
        W.ev_apply.push_back(e);
    }
    if (!W.ev_cgs) TSK_HIP(hipEventCreateWithFlags(&W.ev_cgs, hipEventDisableTiming));
    if (!W.side) TSK_HIP(hipStreamCreateWithFlags(&W.side, hipStreamNonBlocking));
    const hipStream_t s2 = W.side;
    W.m = m;
    W.steps = 0;
    W.ldv = ldv;

    TS* V = W.V.as<TS>();
    double2* H = W.H.as<double2>();
    TS* w = W.w.as<TS>();
    double* scal = W.scal.as<double>();
    RitzResult* rr = W.rr.as<RitzResult>();
    RitzResult* rrh = W.rr_host;
    double* scal_host = reinterpret_cast<double*>(rrh + 1);

    TSK_HIP(hipMemsetAsync(H, 0, size_t(m + 1) * m * sizeof(double2), s));
    TSK_HIP(hipMemsetAsync(rr, 0, sizeof(RitzResult), s));

    // ---- start vector (Algorithm 1: v1 = v / ||v||) ------------------------------
    const TS* x0 = static_cast<const TS*>(v0);
    if (!x0) {
        const int64_t pr = op->physical_reals();
        TSK_TRY(W.phys.ensure(size_t(pr) * 8));
        TSK_TRY(normal_fill(W.phys.as<double>(), pr, seed, s));
        if (op->kind == StateKind::Real32) {
            // FP32 operators take an FP32 physical field: narrow in place (front half)
            TSK_TRY(narrow_to_float(W.phys.as<double>(), W.phys.as<float>(), pr, s));
        }
        TSK_TRY(op->from_physical(W.phys.ptr, w));
        x0 = w;
    }
    int* flag = reinterpret_cast<int*>(scal + 32);
    TSK_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    launch_check_finite<TS>(x0, n, flag, s);
    launch_dot<TS>(V, ldv, 0, x0, n, W.partial.as<double2>(), W.pnrm.as<double>(), s);
    launch_reduce(W.partial.as<double2>(), nblk, 0, W.h.as<double2>(), nullptr, 0, W.pnrm.as<double>(), scal, 0, s);
    TSK_HIP(hipMemcpyAsync(scal_host, scal, 40 * sizeof(double), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    if (*reinterpret_cast<int*>(scal_host + 32) != 0) return fail(TSK_ENONFINITE, "start vector is not finite");
    if (!(scal_host[0] > 0.0)) return fail(TSK_EINVAL, "start vector is zero");
    launch_scale_state<TS>(x0, scal, 0, V, n, s);

    // ---- Arnoldi steps ------------------------------------------------------------------
    tsk_status status = TSK_NOT_CONVERGED;
    int steps = 0;
    TSK_HIP(hipEventRecord(W.ev_apply[0], s));
    TSK_TRY(op->apply(V, w));
    TSK_HIP(hipEventRecord(W.ev_apply[1], s));
    for (int j = 0; j < m; ++j) {
        const int p = j + 1;
        double2* Hcol = H + size_t(m + 1) * j;
        launch_dot<TS>(V, ldv, p, w, n, W.partial.as<double2>(), W.pnrm.as<double>(), s);
        launch_reduce(W.partial.as<double2>(), nblk, p, W.h.as<double2>(), Hcol, 1, W.pnrm.as<double>(), scal, 1, s);
        launch_update<TS>(V, ldv, p, W.h.as<double2>(), w, nullptr, W.w64.ptr, n, true, W.partial.as<double2>(),
                          W.pnrm.as<double>(), s);
        launch_reduce(W.partial.as<double2>(), nblk, p, W.h.as<double2>(), Hcol, 0, nullptr, scal, 0, s);
        launch_update<TS>(V, ldv, p, W.h.as<double2>(), nullptr, W.w64.ptr, W.w64.ptr, n, false,
                          W.partial.as<double2>(), W.pnrm.as<double>(), s);
        launch_finalize(W.pnrm.as<double>(), nblk, scal, 1, Hcol + p, scal + 2, rr, s);
        launch_scale<TS>(W.w64.ptr, scal + 2, V + (j + 1) * ldv, n, s);
        TSK_HIP(hipEventRecord(W.ev_cgs, s));
        // speculative matvec of the next step
        if (j + 1 < m) {
            TSK_HIP(hipEventRecord(W.ev_apply[2 * (j + 1)], s));
            TSK_TRY(op->apply(V + (j + 1) * ldv, w));
            TSK_HIP(hipEventRecord(W.ev_apply[2 * (j + 1) + 1], s));
        }
        // Ritz analysis of H_j on the side stream
        TSK_HIP(hipStreamWaitEvent(s2, W.ev_cgs, 0));
        const int kk = k < p ? k : p;
        TSK_TRY(hess_ritz_launch(H, m + 1, p, scal + 2, 0.0, W.eigZ.as<double2>(), W.eigS.as<double2>(),
                                 W.eigMu.as<double2>(), W.eigY.as<double2>(), W.eigRes.as<double>(), kk, tol,
                                 op->kind == StateKind::Real32 ? kDupRelFp32 : 0.0, W.sel.as<int>(), rr, s2));
        TSK_HIP(hipMemcpyAsync(rrh, rr, sizeof(RitzResult), hipMemcpyDeviceToHost, s2));
        TSK_HIP(hipStreamSynchronize(s2));
        steps = p;
        W.steps = p;
        if (rrh->nonfinite) return fail(TSK_ENONFINITE, "non-finite matvec output or norm at step " + std::to_string(p));
        if (rrh->eig_fail) return fail(TSK_EEIG, "Hessenberg QR did not converge at step " + std::to_string(p));
        if (rrh->breakdown) { status = TSK_BREAKDOWN; break; }
        if (rrh->done && kk == k) { status = TSK_OK; break; }
    }

    // ---- outputs ---------------------------------------------------------------------------
    TSK_HIP(hipStreamSynchronize(s));  // drains a discarded speculative matvec
    double ms_apply = 0.0;
    for (int j = 0; j < steps; ++j) {
        float ms = 0.0f;
        TSK_HIP(hipEventElapsedTime(&ms, W.ev_apply[2 * j], W.ev_apply[2 * j + 1]));
        ms_apply += ms;
    }
    const int nsel = rrh->nsel;
    double* gath = reinterpret_cast<double*>(static_cast<char*>(W.sel.ptr) + gath_off);
    hipLaunchKernelGGL(k_gather_ritz, dim3(1), dim3(128), 0, s, W.eigMu.as<double2>(), W.eigRes.as<double>(),
                       W.sel.as<int>(), nsel, op->T, gath);
    TSK_HIP(hipGetLastError());
    if (ritz && nsel > 0)
        TSK_TRY(ritz_coords_launch(H, m + 1, steps, W.eigMu.as<double2>(), W.sel.as<int>(), nsel,
                                   W.eigY.as<double2>(), s));
    if (ritz && nsel > 0)
        launch_ritz_vectors<TS>(V, ldv, steps, W.eigY.as<double2>(), W.sel.as<int>(), nsel,
                                static_cast<double2*>(ritz), n, s);
    std::vector<double> hbuf(5 * size_t(nsel > 0 ? nsel : 1));
    if (nsel > 0)
        TSK_HIP(hipMemcpyAsync(hbuf.data(), gath, 5 * size_t(nsel) * sizeof(double), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    TSK_HIP(hipGetLastError());
    for (int i = 0; i < k; ++i) {
        bool have = i < nsel;
        if (mu_ri) { mu_ri[2 * i] = have ? hbuf[2 * i] : 0.0; mu_ri[2 * i + 1] = have ? hbuf[2 * i + 1] : 0.0; }
        if (lam_ri) {
            lam_ri[2 * i] = have ? hbuf[2 * nsel + 2 * i] : 0.0;
            lam_ri[2 * i + 1] = have ? hbuf[2 * nsel + 2 * i + 1] : 0.0;
        }
        if (resid) resid[i] = have ? hbuf[4 * nsel + i] : 0.0;
    }
    if (info) {
        info->n_matvec = steps;
        info->n_ritz = nsel;
        info->n_converged = rrh->nconv;
        info->status = status;
        info->beta = rrh->beta;
        info->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->ms_apply = ms_apply;
    }
    return status;
}

}  // namespace

tsk_status arnoldi(Operator* op, int m, int k, double tol, const void* v0, uint64_t seed, double* mu_ri,
                   double* lam_ri, double* resid, void* ritz, tsk_arnoldi_info* info) {
    if (!op->ready()) return fail(TSK_ESTATE, "operator parameters or base flow not set");
    if (k < 1 || m < k || m > kMaxKrylov) return fail(TSK_EINVAL, "need 1 <= k <= m <= 96");
    if (int64_t(m) > op->n) return fail(TSK_EINVAL, "m exceeds the state dimension");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(TSK_EINVAL, "tol must be finite and >= 0");
    switch (op->kind) {
        case StateKind::Complex64x2:
            return arnoldi_t<double2>(op, m, k, tol, v0, seed, mu_ri, lam_ri, resid, ritz, info);
        case StateKind::Real64:
            return arnoldi_t<double>(op, m, k, tol, v0, seed, mu_ri, lam_ri, resid, ritz, info);
        case StateKind::Real32:
            return arnoldi_t<float>(op, m, k, tol, v0, seed, mu_ri, lam_ri, resid, ritz, info);
    }
    return fail(TSK_EINVAL, "unknown state kind");
}

}  // namespace tsk
