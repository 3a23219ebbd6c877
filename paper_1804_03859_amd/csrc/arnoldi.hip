// Arnoldi driver (host orchestration of device kernels) for a batch of
// independent instances advancing in lockstep; a single run is a batch of one.
//
// m-step Arnoldi factorisation M V_m = V_m H_m + beta v_{m+1} e_m^T
// (Sec. 3.2.1, eq. "m-step Arnoldi", Algorithm 1) with every matvec a time
// integration of the linearized equations (Sec. 3, time-stepper approach).
// After each matvec: CGS2 projection and normalisation (krylov.hip), then the
// device Hessenberg QR and wanted-set test (hessenberg.hip), one wavefront per
// instance.  The only device-to-host traffic per step is one 56-byte
// RitzResult per instance, telling the host which instances stop.  Ritz values
// are mapped to lambda = log(mu)/T on the device (principal branch, valid when
// |Im lambda| T < pi/2, the four-samples-per-period rule of Sec. 3.2.1).
//
// Overlap: as soon as v_{j+1} exists, the matvec M v_{j+1} is launched on the
// operator stream while the Ritz analysis of H_j waits for a free analysis
// stream (one wavefront per instance and step, so it barely competes for
// compute units).  Up to kSlots consecutive steps are in flight, each with its
// own output slot; the steps that became ready while every analysis stream
// was busy are analysed together by one launch, so a backlog never waits for
// hardware queues.  The host consumes the analyses in step order and stops an
// instance at the first step whose H_j satisfies the stop test, exactly as a
// check after every step would; work already launched for later steps is
// discarded (neither counted nor used), and its analyses return early once the
// host raises the instance's stop flag.  Batched Navier-Stokes instances share
// one launch per grid size for the matvec; kernels of the Gram-Schmidt and
// Ritz phases index the instance by blockIdx.
#include <array>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

// The worker streams (Ritz analyses; the extra grid-size groups of a batched
// matvec) are shared by every workspace of the process, one set per device,
// created on first use and kept until the process ends.  A process gets 4
// hardware queues by default (GPU_MAX_HW_QUEUES): with a set per operator, a
// run after a few operators had been created put its analyses on the operator
// stream's queue, in front of its matvecs (a 256^2 run took 34 instead of
// 20 ms).  Runs are sequential and wait for these streams at their end, so
// sharing them is safe.
tsk_status analysis_streams(hipStream_t (&out)[ArnoldiWork::kAnaStreams]) {
    static std::mutex mu;
    static std::map<int, std::array<hipStream_t, ArnoldiWork::kAnaStreams>> per_device;
    int dev = 0;
    TSK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = per_device.find(dev);
    if (it == per_device.end()) {
        std::array<hipStream_t, ArnoldiWork::kAnaStreams> st{};
        for (auto& q : st) TSK_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        it = per_device.emplace(dev, st).first;
    }
    for (int a = 0; a < ArnoldiWork::kAnaStreams; ++a) out[a] = it->second[a];
    return TSK_OK;
}

namespace {

__global__ void k_collect(const KryDesc* __restrict__ Dv, int count, RitzResult* __restrict__ dst, int with_scal) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        RitzResult r = *Dv[i].rr;
        if (with_scal) {  // start-vector checks: ||x0||^2 in beta, finite flag in nonfinite
            r.beta = Dv[i].scal[0];
            r.nonfinite = *reinterpret_cast<const int*>(Dv[i].scal + 32);
        }
        dst[i] = r;
    }
}

// RitzResults of the n consecutive slots first, first + 1, ... (mod nslots) of
// the slot tables D (slot t at D + t count) into dst at the same positions:
// one launch per analysis batch.
__global__ void k_collect_slots(const KryDesc* __restrict__ D, int count, int nslots, int first,
                                RitzResult* __restrict__ dst) {
    const int t = (first + int(blockIdx.x)) % nslots;
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[size_t(t) * count + i] = *D[size_t(t) * count + i].rr;
}

// Zero H, the start-vector flag and the RitzResult of every slot table.
__global__ void k_reset(const KryDesc* __restrict__ Dv, int count, int nslots) {
    const KryDesc& d = Dv[blockIdx.x];
    for (int i = threadIdx.x; i < d.ldh * (d.ldh - 1); i += blockDim.x) d.H[i] = cmk<double2>(0.0, 0.0);
    if (threadIdx.x == 0) {
        for (int t = 0; t < nslots; ++t) *Dv[size_t(t) * count + blockIdx.x].rr = RitzResult{};
        *reinterpret_cast<int*>(d.scal + 32) = 0;
        *cgs_counter(d) = 0;
    }
}

// Instance i has stopped: every slot table marks it inactive.
__global__ void k_deactivate(KryDesc* __restrict__ Dv, int count, int nslots, int i) {
    if (threadIdx.x == 0)
        for (int t = 0; t < nslots; ++t) Dv[size_t(t) * count + i].active = 0;
}

template <typename TS> struct WorkType { using A = double; };
template <> struct WorkType<double2> { using A = double2; };

struct Outcome {
    int status = TSK_NOT_CONVERGED;
    int steps = 0;
    bool done = false;
    std::string err;
};

// Workspace of one instance (NS copies of the eigensolver outputs) and its
// descriptor; ritz: optional Ritz-vector output.
template <typename TS>
tsk_status make_desc(Operator* op, int m, int k, int NS, void* ritz, KryDesc& d) {
    using A = typename WorkType<TS>::A;
    ArnoldiWork& W = op->aw;
    const int64_t n = op->n;
    const int64_t ldv = (n + 63) / 64 * 64;
    const int nblk = cgs_blocks(n);
    TSK_TRY(W.V.ensure(size_t(m + 1) * ldv * sizeof(TS)));
    TSK_TRY(W.H.ensure(size_t(m + 1) * m * sizeof(double2)));
    TSK_TRY(W.w.ensure(size_t(n) * sizeof(TS)));
    TSK_TRY(W.w64.ensure(size_t(n) * sizeof(A)));
    TSK_TRY(W.partial.ensure(2 * size_t(nblk) * (m + 1) * sizeof(double2)));
    TSK_TRY(W.pnrm.ensure(2 * size_t(nblk) * sizeof(double)));
    TSK_TRY(W.h.ensure(size_t(m + 1) * sizeof(double2)));
    TSK_TRY(W.scal.ensure(64 * sizeof(double)));
    TSK_TRY(W.eigS.ensure(size_t(NS) * m * m * sizeof(double2)));
    TSK_TRY(W.eigY.ensure(size_t(m) * (k > 0 ? k : 1) * sizeof(double2)));
    TSK_TRY(W.eigMu.ensure(size_t(NS) * m * sizeof(double2)));
    TSK_TRY(W.eigRes.ensure(size_t(NS) * m * sizeof(double)));
    TSK_TRY(W.sel.ensure(size_t(NS) * m * sizeof(int)));
    TSK_TRY(W.out.ensure(5 * size_t(k) * sizeof(double)));
    TSK_TRY(W.rr.ensure(size_t(NS) * sizeof(RitzResult)));
    W.m = m;
    W.steps = 0;
    W.ldv = ldv;
    std::memset(&d, 0, sizeof(d));
    d.V = W.V.ptr;
    d.w = W.w.ptr;
    d.w64 = W.w64.ptr;
    d.H = W.H.as<double2>();
    d.partial = W.partial.as<double2>();
    d.pnrm = W.pnrm.as<double>();
    d.partial2 = d.partial + size_t(nblk) * (m + 1);
    d.pnrm2 = d.pnrm + nblk;
    d.h = W.h.as<double2>();
    d.scal = W.scal.as<double>();
    d.Z = nullptr;
    d.S = W.eigS.as<double2>();
    d.Y = W.eigY.as<double2>();
    d.mu = W.eigMu.as<double2>();
    d.res = W.eigRes.as<double>();
    d.sel = W.sel.as<int>();
    d.rr = W.rr.as<RitzResult>();
    d.ritz = ritz;
    d.out = W.out.as<double>();
    d.ldv = ldv;
    d.n = n;
    d.ldh = m + 1;
    d.nblk = nblk;
    d.active = 1;
    d.dup_rel = op->stop_dup_rel >= 0.0 ? op->stop_dup_rel : op->kind == StateKind::Real32 ? kDupRelFp32 : 0.0;
    d.res_floor = op->stop_res_floor >= 0.0 ? op->stop_res_floor
                                            : op->kind == StateKind::Real32 ? kResFloorFp32 : 0.0;
    d.T = op->T;
    W.Vcur = W.V.ptr;
    return TSK_OK;
}

// Start vector drawn from `seed`: an iid N(0,1) physical field (splitmix64 +
// Box-Muller) projected on the state space, written to the instance's w.
tsk_status seeded_start(Operator* op, uint64_t seed, hipStream_t s, const void** x0) {
    const int64_t pr = op->physical_reals();
    TSK_TRY(op->aw.phys.ensure(size_t(pr) * 8));
    TSK_TRY(normal_fill(op->aw.phys.as<double>(), pr, seed, s));
    if (op->kind == StateKind::Real32) TSK_TRY(narrow_to_float(op->aw.phys.as<double>(), op->aw.phys.as<float>(), pr, s));
    TSK_TRY(op->from_physical(op->aw.phys.ptr, op->aw.w.ptr));
    *x0 = op->aw.w.ptr;
    return TSK_OK;
}

// Reset of the descriptor table D (count instances, nslots slot tables), norm
// and finiteness of the start vectors, then V_0 = x0 / ||x0|| (Algorithm 1).
template <typename TS>
tsk_status normalize_starts(const KryDesc* D, int count, int nslots, int64_t nmax, int nblk_max, ArnoldiWork& L,
                            hipStream_t s) {
    RitzResult* rrh = L.rr_host;
    hipLaunchKernelGGL(k_reset, dim3(count), dim3(256), 0, s, D, count, nslots);
    launch_check_finite<TS>(D, count, nmax, s);
    launch_dot<TS>(D, count, nblk_max, 0, true, s);
    launch_reduce_norm(D, count, 0, s);
    hipLaunchKernelGGL(k_collect, dim3(1), dim3(256), 0, s, D, count, L.batch_rr.as<RitzResult>(), 1);
    TSK_HIP(hipMemcpyAsync(rrh, L.batch_rr.ptr, size_t(count) * sizeof(RitzResult), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {
        if (rrh[i].nonfinite) return fail(TSK_ENONFINITE, "start vector " + std::to_string(i) + " is not finite");
        if (!(rrh[i].beta > 0.0)) return fail(TSK_EINVAL, "start vector " + std::to_string(i) + " is zero");
    }
    launch_scale<TS>(D, count, nmax, -1, s);
    return TSK_OK;
}

// Timing events (two per matvec of up to m + 1 steps), the analysis streams
// with their events, and the device and pinned copies of nrr RitzResults.
tsk_status driver_resources(ArnoldiWork& L, int m, int nrr) {
    constexpr int NS = ArnoldiWork::kSlots;
    while (L.ev_apply.size() < size_t(2 * (m + 1))) {
        hipEvent_t e;
        TSK_HIP(hipEventCreate(&e));
        L.ev_apply.push_back(e);
    }
    for (int t = 0; t < NS; ++t) {
        if (!L.ev_cgs[t]) TSK_HIP(hipEventCreateWithFlags(&L.ev_cgs[t], hipEventDisableTiming));
        if (!L.ev_eig[t]) TSK_HIP(hipEventCreateWithFlags(&L.ev_eig[t], hipEventDisableTiming));
        if (t < ArnoldiWork::kAnaStreams && !L.ev_ana[t])
            TSK_HIP(hipEventCreateWithFlags(&L.ev_ana[t], hipEventDisableTiming));
    }
    if (!L.side[0]) TSK_TRY(analysis_streams(L.side));
    TSK_TRY(L.batch_rr.ensure(size_t(nrr) * sizeof(RitzResult)));
    if (L.rr_host_count < nrr) {
        if (L.rr_host) (void)hipHostFree(L.rr_host);
        L.rr_host = nullptr;
        TSK_HIP(hipHostMalloc((void**)&L.rr_host, size_t(nrr) * sizeof(RitzResult), 0));
        L.rr_host_count = nrr;
    }
    return TSK_OK;
}

// Step j of the factorisation after the matvec w = M v_j: classical
// Gram-Schmidt twice against v_0..v_j (H column j = h1 + h2), beta_j = ||f||,
// H[j+1][j] = beta_j, v_{j+1} = f / beta_j (Algorithm 1 with CGS2).
// pextra: the largest step offset (KryDesc::poff) of the table, 0 in ordinary runs.
template <typename TS>
void cgs2_step(const KryDesc* Dt, int count, int nblk_max, int64_t nmax, int j, hipStream_t s, int pextra = 0) {
    const int p = j + 1;
    const bool fuse = nblk_max <= kFuseFinalMaxBlocks;
    launch_dot<TS>(Dt, count, nblk_max, p, false, s);
    launch_cgs_pass<TS>(Dt, count, nblk_max, p, j, 1, false, s, pextra);  // h1 = V^H w, w -= V h1, dots for pass 2
    launch_cgs_pass<TS>(Dt, count, nblk_max, p, j, 2, fuse, s, pextra);   // h2, w -= V h2, squared norm
    if (!fuse) launch_scale_final<TS>(Dt, count, nmax, j, s);             // beta, H[j+1][j], flags, v_{j+1}
}

// svd = false: Arnoldi on M (Algorithm 1).  svd = true: Lanczos on M^dagger M
// (Sec. 3.3.2): each step is a forward then an adjoint integration, the Ritz
// analysis is the symmetric tridiagonal solver (the same CGS2 against every
// previous vector serves as full reorthogonalisation).
template <typename TS>
tsk_status arnoldi_t(Operator* const* ops, int count, int m, int k, double tol, const void* const* v0s,
                     const uint64_t* seeds, double* mu_ri, double* lam_ri, double* resid, void* const* ritz,
                     tsk_arnoldi_info* infos, bool svd, const BatchRestart* rs) {
    auto t0 = std::chrono::steady_clock::now();
    Operator* lead = ops[0];
    const hipStream_t s = lead->stream;
    ArnoldiWork& L = lead->aw;
    constexpr int NS = ArnoldiWork::kSlots;
    constexpr bool kRealH = !std::is_same<TS, double2>::value;  // real operators: real Hessenberg QR

    // ---- per-instance workspace and descriptors ------------------------------------
    std::vector<KryDesc> Dh(count);
    int64_t nmax = 0;
    int nblk_max = 0;
    for (int i = 0; i < count; ++i) {
        TSK_TRY(make_desc<TS>(ops[i], m, k, NS, (ritz && ritz[i]) ? ritz[i] : nullptr, Dh[i]));
        if (svd) TSK_TRY(ops[i]->aw.tmp.ensure(ops[i]->state_bytes()));
        nmax = std::max(nmax, ops[i]->n);
        nblk_max = std::max(nblk_max, Dh[i].nblk);
    }
    TSK_TRY(driver_resources(L, m, NS * count));
    RitzResult* rrh = L.rr_host;
    // stop flags (coherent pinned memory, read by the running analyses): raised by
    // the host when an instance finishes, so the analyses of its discarded later
    // steps end early; every side-stream reader of the previous run has finished
    if (L.stop_count < count) {
        if (L.stop_host) (void)hipHostFree(L.stop_host);
        L.stop_host = nullptr;
        L.stop_count = 0;
        TSK_HIP(hipHostMalloc((void**)&L.stop_host, size_t(count) * sizeof(int),
                              hipHostMallocMapped | hipHostMallocCoherent));
        L.stop_count = count;
    }
    int* stop_dev = nullptr;
    TSK_HIP(hipHostGetDevicePointer((void**)&stop_dev, L.stop_host, 0));
    for (int i = 0; i < count; ++i) {
        __atomic_store_n(&L.stop_host[i], 0, __ATOMIC_RELEASE);
        Dh[i].stop = stop_dev + i;
    }
    // slot tables: identical except for the eigensolver outputs
    std::vector<KryDesc> Dall(size_t(NS) * count);
    for (int t = 0; t < NS; ++t)
        for (int i = 0; i < count; ++i) {
            KryDesc d = Dh[i];
            ArnoldiWork& W = ops[i]->aw;
            d.S = W.eigS.as<double2>() + size_t(t) * m * m;
            d.mu = W.eigMu.as<double2>() + size_t(t) * m;
            d.res = W.eigRes.as<double>() + size_t(t) * m;
            d.sel = W.sel.as<int>() + size_t(t) * m;
            d.rr = W.rr.as<RitzResult>() + t;
            Dall[size_t(t) * count + i] = d;
        }
    for (int i = 0; i < count; ++i) Dh[i] = Dall[i];

    // ---- start vectors (Algorithm 1: v1 = v / ||v||) -----------------------------------
    for (int i = 0; i < count; ++i) {
        const void* x0 = (v0s && v0s[i]) ? v0s[i] : nullptr;
        if (!x0) TSK_TRY(seeded_start(ops[i], seeds ? seeds[i] : uint64_t(i), s, &x0));
        Dh[i].x0 = x0;
    }
    for (int t = 0; t < NS; ++t)
        for (int i = 0; i < count; ++i) Dall[size_t(t) * count + i].x0 = Dh[i].x0;
    TSK_TRY(L.batch_desc.ensure(size_t(NS) * count * sizeof(KryDesc)));
    KryDesc* D = L.batch_desc.as<KryDesc>();
    auto table = [&](int t) { return D + size_t(t) * count; };
    TSK_HIP(hipMemcpyAsync(D, Dall.data(), size_t(NS) * count * sizeof(KryDesc), hipMemcpyHostToDevice, s));
    TSK_TRY(normalize_starts<TS>(D, count, NS, nmax, nblk_max, L, s));

    // ---- matvec of step j for every active instance --------------------------------------
    KolmoBatchPtr kb;
    bool all_kolmo = true;
    for (int i = 0; i < count; ++i) all_kolmo = all_kolmo && kolmo_parallel(ops[i]);
    // a single instance with the Bloch-sector stepper calls its own matvec
    const bool own = count == 1 && (kolmo_bloch(ops[0]) || kolmo_couple(ops[0]));
    if (all_kolmo && !svd && !own) TSK_TRY(kolmo_batch_plan(ops, count, Dh.data(), D, &kb));
    CgleBatchPtr cb;
    if (count > 1 && is_cgle(ops[0])) TSK_TRY(cgle_batch_plan(ops, count, Dh.data(), svd, &cb));
    std::vector<Outcome> oc(count);
    auto matvec = [&](int j) -> tsk_status {
        if (kb) return kolmo_batch_matvec(kb.get(), j, s);
        if (cb) return cgle_batch_matvec(cb.get(), j, s);
        for (int i = 0; i < count; ++i) {
            if (oc[i].done) continue;
            const TS* vj = static_cast<TS*>(Dh[i].V) + j * Dh[i].ldv;
            if (svd) {  // M^dagger M v_j: forward, then adjoint integration
                TSK_TRY(ops[i]->apply(vj, ops[i]->aw.tmp.ptr));
                TSK_TRY(ops[i]->apply_adjoint(ops[i]->aw.tmp.ptr, Dh[i].w));
            } else {
                TSK_TRY(ops[i]->apply(vj, Dh[i].w));
            }
        }
        return TSK_OK;
    };

    // ---- Arnoldi steps ------------------------------------------------------------------------
    // enqueue(j): CGS2 of step j (output slot j % NS) and the speculative matvec
    // of step j+1 on the operator stream; step j then waits in `ready` for its
    // Ritz analysis.  launch_ready(): when one of the kAnaStreams analysis
    // streams is idle, all ready steps go to it in one launch (one workgroup
    // per step and instance), followed by their collection and copy to the
    // host.  Analyses are consumed in step order; a new step is enqueued when
    // the analyses are consumed, or, while fewer than NS steps are in flight,
    // as soon as the operator stream has finished the matvec before the last
    // one it was given (one step always queued behind the running matvec).
    constexpr int NA = ArnoldiWork::kAnaStreams;
    // Matvec timing: an event pair around every kTimeEvery-th matvec (the first
    // included); ms_apply is their mean duration times the matvecs run.  A
    // timing event record costs about 3.4 us of operator-stream time between
    // dependent kernels, while the matvec's duration hardly varies: timing
    // every 32nd instead of every 8th matvec made 128^2 FP64 runs 5.86 -> 5.62
    // ms and 256^2 FP64 solves 5.75 -> 5.58 ms in interleaved runs.
    constexpr int kTimeEvery = 32;
    static_assert(NS <= StepSet::kMax, "a batch holds every step in flight");
    // a batch of grid-size groups runs its extra groups on worker streams 1 and 2;
    // its analyses then use stream 0 only, so the operator's stream and the three
    // worker streams stay within the 4 hardware queues
    const int na_use = kb && kolmo_batch_groups(kb.get()) > 1 ? 1 : NA;
    std::vector<int> final_slot(count, 0);
    std::deque<int> pend, ready;
    int next = 0, steps_run = 0, remaining = count;
    bool ana_used[NA] = {};  // analysis stream a has a batch recorded in ev_ana[a]
    int batch_last[NS] = {};  // per slot: the last step of the batch that analyses it
    auto enqueue = [&](int j) -> tsk_status {
        const int t = j % NS;
        cgs2_step<TS>(table(t), count, nblk_max, nmax, j, s);
        TSK_HIP(hipEventRecord(L.ev_cgs[t], s));
        if (j + 1 < m) {
            const bool timed = (j + 1) % kTimeEvery == 0;
            if (timed) TSK_HIP(hipEventRecord(L.ev_apply[2 * (j + 1)], s));
            TSK_TRY(matvec(j + 1));
            if (timed) TSK_HIP(hipEventRecord(L.ev_apply[2 * (j + 1) + 1], s));
        }
        ready.push_back(j);
        return TSK_OK;
    };
    auto launch_ready = [&]() -> tsk_status {
        if (ready.empty()) return TSK_OK;
        int a = -1;
        for (int c = 0; c < na_use && a < 0; ++c) {
            if (!ana_used[c]) { a = c; break; }
            const hipError_t q = hipEventQuery(L.ev_ana[c]);
            if (q == hipSuccess) a = c;
            else if (q != hipErrorNotReady) TSK_HIP(q);
        }
        if (a < 0) return TSK_OK;
        const hipStream_t st = L.side[a];
        StepSet ss{};
        const int n = int(ready.size());
        for (int i = 0; i < n; ++i) {
            ss.tab[i] = table(ready[i] % NS);
            ss.p[i] = ready[i] + 1;
        }
        // the Gram-Schmidt of the newest step implies that of the older ones (one stream)
        TSK_HIP(hipStreamWaitEvent(st, L.ev_cgs[ready.back() % NS], 0));
        TSK_TRY(ritz_steps_launch(ss, n, count, k, tol, svd, kRealH, st));
        // one collection kernel and at most two copies (the slot range may wrap) per batch
        const int t0 = ready.front() % NS;
        hipLaunchKernelGGL(k_collect_slots, dim3(n), dim3(256), 0, st, table(0), count, NS, t0,
                           L.batch_rr.as<RitzResult>());
        const int n1 = std::min(n, NS - t0);
        TSK_HIP(hipMemcpyAsync(rrh + size_t(t0) * count, L.batch_rr.as<RitzResult>() + size_t(t0) * count,
                               size_t(n1) * count * sizeof(RitzResult), hipMemcpyDeviceToHost, st));
        if (n > n1)
            TSK_HIP(hipMemcpyAsync(rrh, L.batch_rr.as<RitzResult>(), size_t(n - n1) * count * sizeof(RitzResult),
                                   hipMemcpyDeviceToHost, st));
        // one event per batch, recorded in its last step's slot: that slot is reused only
        // after every step up to it has been consumed
        for (int i = 0; i < n; ++i) batch_last[ready[i] % NS] = ready.back();
        TSK_HIP(hipEventRecord(L.ev_eig[ready.back() % NS], st));
        TSK_HIP(hipEventRecord(L.ev_ana[a], st));
        ana_used[a] = true;
        for (int i = 0; i < n; ++i) pend.push_back(ready[i]);
        ready.clear();
        return TSK_OK;
    };
    auto consume = [&](int j) {
        const int p = j + 1, t = j % NS, kk = k < p ? k : p;
        steps_run = p;
        for (int i = 0; i < count; ++i) {
            if (oc[i].done) continue;
            oc[i].steps = p;
            final_slot[i] = t;
            const RitzResult& r = rrh[size_t(t) * count + i];
            int st = 0;
            if (r.nonfinite) { st = TSK_ENONFINITE; oc[i].err = "non-finite matvec output or norm"; }
            else if (r.eig_fail) { st = TSK_EEIG; oc[i].err = "Hessenberg QR did not converge"; }
            else if (r.breakdown) st = TSK_BREAKDOWN;
            else if (r.done && kk == k) st = TSK_OK;
            else continue;
            oc[i].status = st;
            oc[i].done = true;
            __atomic_store_n(&L.stop_host[i], 1, __ATOMIC_RELEASE);
            --remaining;
            hipLaunchKernelGGL(k_deactivate, dim3(1), dim3(64), 0, s, D, count, NS, i);
        }
    };
    TSK_HIP(hipEventRecord(L.ev_apply[0], s));
    TSK_TRY(matvec(0));
    TSK_HIP(hipEventRecord(L.ev_apply[1], s));
    TSK_TRY(enqueue(next++));
    while (!pend.empty() || !ready.empty()) {
        TSK_TRY(launch_ready());
        if (!pend.empty()) {
            const int jo = pend.front();
            const hipError_t q = hipEventQuery(L.ev_eig[batch_last[jo % NS] % NS]);
            if (q == hipSuccess) {
                pend.pop_front();
                consume(jo);
                if (remaining == 0) break;
                if (pend.empty() && ready.empty() && next < m) TSK_TRY(enqueue(next++));
                continue;
            }
            if (q != hipErrorNotReady) TSK_HIP(q);
        }
        if (next < m && int(pend.size() + ready.size()) < NS) {
            // one step queued ahead: step `next` (its Gram-Schmidt and the matvec
            // after it) goes behind its own matvec as soon as that matvec can start,
            // i.e. once the Gram-Schmidt of step next - 1 has finished, so the
            // operator stream never waits for the host.  Queueing three steps ahead
            // did not help; one step ahead keeps the fewest discarded matvecs.
            const hipError_t qm = next < 1 ? hipSuccess : hipEventQuery(L.ev_cgs[(next - 1) % NS]);
            if (qm == hipSuccess) {
                TSK_TRY(enqueue(next++));
                continue;
            }
            if (qm != hipErrorNotReady) TSK_HIP(qm);
        }
        std::this_thread::yield();
    }
    for (int a = 0; a < NA; ++a) TSK_HIP(hipStreamSynchronize(L.side[a]));  // discarded analyses

    // ---- outputs --------------------------------------------------------------------------------
    TSK_HIP(hipStreamSynchronize(s));  // drains discarded speculative matvecs
    double ms_apply = 0.0;
    {
        int nt = 0;
        for (int j = 0; j < steps_run; j += kTimeEvery) {
            float ms = 0.0f;
            TSK_HIP(hipEventElapsedTime(&ms, L.ev_apply[2 * j], L.ev_apply[2 * j + 1]));
            ms_apply += ms;
            ++nt;
        }
        if (nt > 0) ms_apply = ms_apply / nt * steps_run;
    }
    int pmax = 1;
    for (int i = 0; i < count; ++i) {
        Dh[i] = Dall[size_t(final_slot[i]) * count + i];  // the analysis of the final step
        Dh[i].steps = oc[i].steps;
        Dh[i].active = 1;
        if (svd) Dh[i].Y = Dh[i].S;  // the tridiagonal solver left the unit Ritz coordinates there
        ops[i]->aw.steps = oc[i].steps;
        pmax = std::max(pmax, oc[i].steps);
    }

    // ---- batched restart phase (Sec. 3.2.2): the instances not converged at order m ------------
    // contract to the Krylov-Schur form of their kept Ritz values (one wavefront each,
    // the kernel of tsk_krylov_schur), rotate their bases and expand again in
    // lockstep, instance i from its own kept order p_i (its step = the batch step
    // + p_i); convergence is tested at order m, as in Krylov-Schur.
    std::vector<int> extra_mv(count, 0), n_restarts(count, 0), kept_last(count, 0);
    if (rs && !svd && kRealH) {
        std::vector<int> R;
        for (int i = 0; i < count; ++i)
            if (oc[i].status == TSK_NOT_CONVERGED && oc[i].steps == m) R.push_back(i);
        std::vector<void*> Vcur(count, nullptr), Valt(count, nullptr);
        std::vector<KryDesc> DR;
        int64_t nmax_r = 0;
        int nblk_max_r = 0;
        for (int i : R) {
            ArnoldiWork& W = ops[i]->aw;
            TSK_TRY(W.V2.ensure(size_t(m + 1) * W.ldv * sizeof(TS)));
            TSK_TRY(W.ksW.ensure(size_t(m) * m * sizeof(double)));
            Vcur[i] = W.V.ptr;
            Valt[i] = W.V2.ptr;
            KryDesc d = Dh[i];
            d.ksW = W.ksW.as<double>();
            d.ks_delta = rs->delta;
            d.ks_pmax = rs->pmax;
            d.poff = 0;
            d.steps = m;
            DR.push_back(d);
            nmax_r = std::max(nmax_r, ops[i]->n);
            nblk_max_r = std::max(nblk_max_r, d.nblk);
        }
        if (!R.empty()) {
            TSK_TRY(L.ks_desc.ensure(R.size() * sizeof(KryDesc)));
            TSK_TRY(L.batch_rr.ensure(std::max(size_t(NS) * count, R.size()) * sizeof(RitzResult)));
        }
        KryDesc* DRd = L.ks_desc.as<KryDesc>();
        int cycle = 0;
        while (!R.empty()) {
            const int nr = int(R.size());
            TSK_HIP(hipMemcpyAsync(DRd, DR.data(), nr * sizeof(KryDesc), hipMemcpyHostToDevice, s));
            const int contract = cycle < rs->max_restarts ? 1 : 0;
            TSK_TRY(ks_contract_launch(DRd, m, k, tol, contract, s, nr));
            hipLaunchKernelGGL(k_collect, dim3(1), dim3(256), 0, s, DRd, nr, L.batch_rr.as<RitzResult>(), 0);
            TSK_HIP(hipMemcpyAsync(rrh, L.batch_rr.ptr, size_t(nr) * sizeof(RitzResult), hipMemcpyDeviceToHost, s));
            TSK_HIP(hipStreamSynchronize(s));
            std::vector<int> keepR;
            std::vector<KryDesc> keepD;
            std::vector<int> kp;
            for (int q = 0; q < nr; ++q) {
                const int i = R[q];
                const RitzResult r = rrh[q];
                KryDesc d = DR[q];
                d.poff = 0;
                int st = -100;
                if (r.nonfinite) { st = TSK_ENONFINITE; oc[i].err = "non-finite matvec output or norm"; }
                else if (r.eig_fail == 1) { st = TSK_EEIG; oc[i].err = "Hessenberg QR did not converge"; }
                else if (r.eig_fail == 2) { st = TSK_EEIG; oc[i].err = "Schur reordering left no room to expand"; }
                else if (r.bd_step) {
                    // happy breakdown during the last expansion: exact Ritz pairs of that order
                    d.steps = r.bd_step;
                    TSK_HIP(hipMemcpyAsync(DRd + q, &d, sizeof(KryDesc), hipMemcpyHostToDevice, s));
                    TSK_TRY(hess_ritz_launch(DRd + q, 1, r.bd_step, std::min(k, r.bd_step), tol, false, s, true));
                    TSK_HIP(hipStreamSynchronize(s));
                    st = TSK_BREAKDOWN;
                } else if (r.done) st = TSK_OK;
                else if (!contract) st = TSK_NOT_CONVERGED;
                if (st != -100) {
                    oc[i].status = st;
                    Dh[i] = d;
                    Dh[i].V = Vcur[i];
                    Dh[i].active = 1;
                    ops[i]->aw.Vcur = Vcur[i];
                    ops[i]->aw.steps = d.steps;
                    continue;
                }
                keepR.push_back(i);
                keepD.push_back(d);
                kp.push_back(r.kept);
            }
            if (keepR.empty()) break;
            // V_p = V_m W, v_{p+1} = v_{m+1} into the other buffer; expansion inputs and offsets
            std::vector<const void*> xb(count, nullptr);
            std::vector<int> jm(count, 0);
            int pmin = m, pext = 0;
            for (size_t q = 0; q < keepR.size(); ++q) {
                const int i = keepR[q], p_i = kp[q];
                ArnoldiWork& W = ops[i]->aw;
                launch_rotate<TS>(Vcur[i], Valt[i], keepD[q].ksW, ops[i]->n, W.ldv, m, p_i, s);
                std::swap(Vcur[i], Valt[i]);
                keepD[q].V = Vcur[i];
                keepD[q].poff = p_i;
                xb[i] = static_cast<const TS*>(Vcur[i]) + size_t(p_i) * W.ldv;
                jm[i] = m - p_i;
                pmin = std::min(pmin, p_i);
                pext = std::max(pext, p_i);
                extra_mv[i] += m - p_i;
                ++n_restarts[i];
                kept_last[i] = p_i;
            }
            R = keepR;
            DR = keepD;
            const int nr2 = int(R.size());
            TSK_HIP(hipMemcpyAsync(DRd, DR.data(), nr2 * sizeof(KryDesc), hipMemcpyHostToDevice, s));
            // the matvecs of the restarting instances only: a batch plan of their own
            // (instance q of the plan is R[q], its flags in the restart table)
            KolmoBatchPtr kbr;
            if (kb) {
                std::vector<Operator*> opsR;
                std::vector<const void*> xbr;
                std::vector<int> jmr;
                for (int i : R) {
                    opsR.push_back(ops[i]);
                    xbr.push_back(xb[i]);
                    jmr.push_back(jm[i]);
                }
                TSK_TRY(kolmo_batch_plan(opsR.data(), nr2, DR.data(), DRd, &kbr));
                TSK_TRY(kolmo_batch_set_inputs(kbr.get(), xbr.data(), jmr.data(), s));
            }
            const int G = m - pmin;
            // the whole expansion of the cycle (G lockstep steps of matvec and
            // Gram-Schmidt, the offsets fixed for the cycle) of a batch with one
            // matvec launch per step is one graph, captured on the idle worker
            // stream 0 and launched once on the operator's stream; other batches
            // (matvec groups forked to worker streams, or the operators' own matvecs
            // on their streams) launch directly
            // timed: HIP events around every matvec (direct launches only: event
            // nodes of a captured graph do not bracket its kernel nodes)
            auto expand = [&](hipStream_t es, bool timed) -> tsk_status {
                for (int g = 0; g < G; ++g) {
                    if (timed) TSK_HIP(hipEventRecord(L.ev_apply[2 * g], es));
                    if (kbr) {
                        TSK_TRY(kolmo_batch_matvec(kbr.get(), g, es));
                    } else {
                        for (int q = 0; q < nr2; ++q) {
                            const int i = R[q];
                            if (g < jm[i])
                                TSK_TRY(ops[i]->apply(static_cast<const TS*>(xb[i]) + size_t(g) * ops[i]->aw.ldv,
                                                      DR[q].w));
                        }
                    }
                    if (timed) TSK_HIP(hipEventRecord(L.ev_apply[2 * g + 1], es));
                    cgs2_step<TS>(DRd, nr2, nblk_max_r, nmax_r, g, es, pext);
                }
                return TSK_OK;
            };
            const bool graphed = kbr && kolmo_batch_groups(kbr.get()) <= 1;
            if (graphed) {
                const hipStream_t cs = L.side[0];
                TSK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                const tsk_status est = expand(cs, false);
                hipGraph_t graph = nullptr;
                const hipError_t ce = hipStreamEndCapture(cs, &graph);
                TSK_TRY(est);
                TSK_HIP(ce);
                hipGraphExec_t exec = nullptr;
                const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                const hipError_t le = ie == hipSuccess ? hipGraphLaunch(exec, s) : ie;
                const hipError_t se = hipStreamSynchronize(s);
                if (exec) (void)hipGraphExecDestroy(exec);
                (void)hipGraphDestroy(graph);
                TSK_HIP(le);
                TSK_HIP(se);
            } else {
                TSK_TRY(expand(s, true));
                TSK_HIP(hipStreamSynchronize(s));
                for (int g = 0; g < G; ++g) {
                    float ms = 0.0f;
                    TSK_HIP(hipEventElapsedTime(&ms, L.ev_apply[2 * g], L.ev_apply[2 * g + 1]));
                    ms_apply += ms;
                }
            }
            for (KryDesc& d : DR) d.poff = 0;  // order m again: the contraction reads H_m
            ++cycle;
        }
        for (int i = 0; i < count; ++i) pmax = std::max(pmax, Dh[i].steps);
    }
    TSK_HIP(hipMemcpyAsync(D, Dh.data(), size_t(count) * sizeof(KryDesc), hipMemcpyHostToDevice, s));
    bool any_ritz = false;
    for (int i = 0; i < count; ++i) any_ritz = any_ritz || Dh[i].ritz;
    if (any_ritz) {
        if (!svd) TSK_TRY(ritz_coords_launch(D, count, pmax, k, s));
        launch_ritz_vectors<TS>(D, count, nmax, k, s);
    }
    launch_gather(D, count, k, s);
    std::vector<double> hout(5 * size_t(k) * count);
    for (int i = 0; i < count; ++i)
        TSK_HIP(hipMemcpyAsync(hout.data() + 5 * size_t(k) * i, Dh[i].out, 5 * size_t(k) * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(k_collect, dim3(1), dim3(256), 0, s, D, count, L.batch_rr.as<RitzResult>(), 0);
    TSK_HIP(hipMemcpyAsync(rrh, L.batch_rr.ptr, size_t(count) * sizeof(RitzResult), hipMemcpyDeviceToHost, s));
    TSK_HIP(hipStreamSynchronize(s));
    TSK_HIP(hipGetLastError());
    const double ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < count; ++i) {
        const double* o = hout.data() + 5 * size_t(k) * i;
        const bool ok = oc[i].status >= 0;
        for (int q = 0; q < k; ++q) {
            if (mu_ri) { mu_ri[2 * k * i + 2 * q] = ok ? o[2 * q] : 0.0; mu_ri[2 * k * i + 2 * q + 1] = ok ? o[2 * q + 1] : 0.0; }
            if (lam_ri) {
                lam_ri[2 * k * i + 2 * q] = ok ? o[2 * k + 2 * q] : 0.0;
                lam_ri[2 * k * i + 2 * q + 1] = ok ? o[2 * k + 2 * q + 1] : 0.0;
            }
            if (resid) resid[k * i + q] = ok ? o[4 * k + q] : 0.0;
        }
        if (rs && rs->infos) {
            tsk_ks_info& f = rs->infos[i];
            f.n_matvec = oc[i].steps + extra_mv[i];
            f.n_restarts = n_restarts[i];
            f.n_ritz = ok ? rrh[i].nsel : 0;
            f.n_converged = ok ? rrh[i].nconv : 0;
            f.status = oc[i].status;
            f.kept_last = kept_last[i];
            f.beta = rrh[i].beta;
            f.ms_total = ms_total;
            f.ms_apply = ms_apply;
        }
        if (infos) {
            tsk_arnoldi_info& f = infos[i];
            f.n_matvec = oc[i].steps + extra_mv[i];
            f.n_ritz = ok ? rrh[i].nsel : 0;
            f.n_converged = ok ? rrh[i].nconv : 0;
            f.status = oc[i].status;
            f.beta = rrh[i].beta;
            f.ms_total = ms_total;
            f.ms_apply = ms_apply;
        }
    }
    if (count == 1 && oc[0].status < 0) return fail(tsk_status(oc[0].status), oc[0].err + " at step " + std::to_string(oc[0].steps));
    return count == 1 ? tsk_status(oc[0].status) : TSK_OK;
}


// ---- Krylov-Schur driver (Sec. 3.2.2) -------------------------------------------------------
// Expansion: Arnoldi steps j0..m-1 (matvec + CGS2) enqueued without host
// synchronisation.  At order m, one kernel analyses H_m (Ritz pairs, residuals,
// stop test; convergence is tested only at full order, steps 2 and 6 of the
// method) and, when the test fails, contracts it to an Arnoldi factorisation
// of order p (hessenberg.hip); the host reads the 56-byte result, rotates the
// basis into the second buffer (V_p = V_m W, v_{p+1} = v_{m+1}) and expands
// again from j0 = p.  A breakdown during an expansion (sticky bd_step) ends the
// run with the exact Ritz pairs of that order.
template <typename TS>
tsk_status krylov_schur_t(Operator* op, int m, int k, double tol, double delta, int pmax, int max_restarts,
                          const void* v0, uint64_t seed, double* mu_ri, double* lam_ri, double* resid, void* ritz,
                          tsk_ks_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    const hipStream_t s = op->stream;
    ArnoldiWork& L = op->aw;
    KryDesc d;
    TSK_TRY(make_desc<TS>(op, m, k, 1, ritz, d));
    TSK_TRY(L.V2.ensure(size_t(m + 1) * d.ldv * sizeof(TS)));
    TSK_TRY(L.ksW.ensure(size_t(m) * m * sizeof(double)));
    d.ksW = L.ksW.as<double>();
    d.ks_delta = delta;
    d.ks_pmax = pmax;
    TSK_TRY(driver_resources(L, m, 1));
    RitzResult* rrh = L.rr_host;
    if (!v0) TSK_TRY(seeded_start(op, seed, s, &v0));
    d.x0 = v0;
    TSK_TRY(L.batch_desc.ensure(sizeof(KryDesc)));
    KryDesc* D = L.batch_desc.as<KryDesc>();
    TSK_HIP(hipMemcpyAsync(D, &d, sizeof(KryDesc), hipMemcpyHostToDevice, s));
    const int64_t n = op->n;
    TSK_TRY(normalize_starts<TS>(D, 1, 1, n, d.nblk, L, s));

    auto collect = [&]() -> tsk_status {
        hipLaunchKernelGGL(k_collect, dim3(1), dim3(64), 0, s, D, 1, L.batch_rr.as<RitzResult>(), 0);
        TSK_HIP(hipMemcpyAsync(rrh, L.batch_rr.ptr, sizeof(RitzResult), hipMemcpyDeviceToHost, s));
        TSK_HIP(hipStreamSynchronize(s));
        return TSK_OK;
    };
    void* Vcur = L.V.ptr;
    void* Valt = L.V2.ptr;
    int j0 = 0, n_matvec = 0, restarts = 0, order = m, kept_last = 0;
    double ms_apply = 0.0;
    int status = TSK_NOT_CONVERGED;
    std::string err;
    while (true) {
        for (int j = j0; j < m; ++j) {  // expansion (step 1, or step 5 after a contraction)
            TSK_HIP(hipEventRecord(L.ev_apply[2 * j], s));
            TSK_TRY(op->apply(static_cast<const TS*>(Vcur) + j * d.ldv, d.w));
            TSK_HIP(hipEventRecord(L.ev_apply[2 * j + 1], s));
            cgs2_step<TS>(D, 1, d.nblk, n, j, s);
        }
        const int contract = restarts < max_restarts ? 1 : 0;
        TSK_TRY(ks_contract_launch(D, m, k, tol, contract, s));
        TSK_TRY(collect());
        for (int j = j0; j < m; ++j) {
            float ms = 0.0f;
            TSK_HIP(hipEventElapsedTime(&ms, L.ev_apply[2 * j], L.ev_apply[2 * j + 1]));
            ms_apply += ms;
        }
        RitzResult r = rrh[0];
        if (r.bd_step) {  // happy breakdown at order bd_step: exact Ritz pairs of that order
            order = r.bd_step;
            n_matvec += order - j0;
            TSK_TRY(hess_ritz_launch(D, 1, order, std::min(k, order), tol, false, s, true));
            TSK_TRY(collect());
            r = rrh[0];
            if (r.nonfinite) { status = TSK_ENONFINITE; err = "non-finite matvec output or norm"; }
            else if (r.eig_fail) { status = TSK_EEIG; err = "Hessenberg QR did not converge"; }
            else status = TSK_BREAKDOWN;
            break;
        }
        n_matvec += m - j0;
        if (r.nonfinite) { status = TSK_ENONFINITE; err = "non-finite matvec output or norm"; break; }
        if (r.eig_fail == 1) { status = TSK_EEIG; err = "Hessenberg QR did not converge"; break; }
        if (r.eig_fail == 2) { status = TSK_EEIG; err = "Schur reordering left no room to expand"; break; }
        if (r.done) { status = TSK_OK; break; }
        if (!contract) break;
        // step 4: V_p = V_m W, v_{p+1} = v_{m+1}, in the other buffer
        const int kp = r.kept;
        launch_rotate<TS>(Vcur, Valt, d.ksW, n, d.ldv, m, kp, s);
        std::swap(Vcur, Valt);
        d.V = Vcur;
        TSK_HIP(hipMemcpyAsync(D, &d, sizeof(KryDesc), hipMemcpyHostToDevice, s));
        j0 = kp;
        kept_last = kp;
        ++restarts;
    }
    L.Vcur = Vcur;
    L.steps = order;
    if (status < 0) return fail(tsk_status(status), err + " after " + std::to_string(n_matvec) + " matvecs");

    // ---- outputs (Ritz pairs of the final factorisation of order `order`) ------------------
    d.steps = order;
    TSK_HIP(hipMemcpyAsync(D, &d, sizeof(KryDesc), hipMemcpyHostToDevice, s));
    if (ritz) {
        TSK_TRY(ritz_coords_launch(D, 1, order, k, s));
        launch_ritz_vectors<TS>(D, 1, n, k, s);
    }
    launch_gather(D, 1, k, s);
    std::vector<double> hout(5 * size_t(k));
    TSK_HIP(hipMemcpyAsync(hout.data(), d.out, 5 * size_t(k) * sizeof(double), hipMemcpyDeviceToHost, s));
    TSK_TRY(collect());
    const RitzResult& r = rrh[0];
    const double ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < k; ++q) {
        const bool have = q < r.nsel;
        if (mu_ri) {
            mu_ri[2 * q] = have ? hout[2 * q] : 0.0;
            mu_ri[2 * q + 1] = have ? hout[2 * q + 1] : 0.0;
        }
        if (lam_ri) {
            lam_ri[2 * q] = have ? hout[2 * k + 2 * q] : 0.0;
            lam_ri[2 * q + 1] = have ? hout[2 * k + 2 * q + 1] : 0.0;
        }
        if (resid) resid[q] = have ? hout[4 * k + q] : 0.0;
    }
    if (info) {
        info->n_matvec = n_matvec;
        info->n_restarts = restarts;
        info->n_ritz = r.nsel;
        info->n_converged = r.nconv;
        info->status = status;
        info->kept_last = kept_last;
        info->beta = r.beta;
        info->ms_total = ms_total;
        info->ms_apply = ms_apply;
    }
    return tsk_status(status);
}

}  // namespace

tsk_status arnoldi_batch(Operator* const* ops, int count, int m, int k, double tol, const void* const* v0s,
                         const uint64_t* seeds, double* mu_ri, double* lam_ri, double* resid, void* const* ritz,
                         tsk_arnoldi_info* infos, bool svd, const BatchRestart* rs) {
    if (count < 1 || !ops) return fail(TSK_EINVAL, "empty batch");
    if (k < 1 || m < k || m > kMaxKrylov) return fail(TSK_EINVAL, "need 1 <= k <= m <= 96");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(TSK_EINVAL, "tol must be finite and >= 0");
    for (int i = 0; i < count; ++i) {
        if (!ops[i]) return fail(TSK_EINVAL, "null operator in batch");
        if (!ops[i]->ready()) return fail(TSK_ESTATE, "operator parameters or base flow not set");
        if (int64_t(m) > ops[i]->n) return fail(TSK_EINVAL, "m exceeds the state dimension");
        if (ops[i]->kind != ops[0]->kind) return fail(TSK_EINVAL, "a batch must share one state type");
        if (ops[i]->stream != ops[0]->stream) return fail(TSK_EINVAL, "batch members must share one stream");
        for (int q = 0; q < i; ++q)
            if (ops[q] == ops[i]) return fail(TSK_EINVAL, "an operator appears twice in the batch");
        if (svd && !ops[i]->has_adjoint())
            return fail(TSK_EINVAL, std::string("no adjoint propagator for this ") + ops[i]->name() + " operator");
    }
    switch (ops[0]->kind) {
        case StateKind::Complex64x2:
            return arnoldi_t<double2>(ops, count, m, k, tol, v0s, seeds, mu_ri, lam_ri, resid, ritz, infos, svd, rs);
        case StateKind::Real64:
            return arnoldi_t<double>(ops, count, m, k, tol, v0s, seeds, mu_ri, lam_ri, resid, ritz, infos, svd, rs);
        case StateKind::Real32:
            return arnoldi_t<float>(ops, count, m, k, tol, v0s, seeds, mu_ri, lam_ri, resid, ritz, infos, svd, rs);
    }
    return fail(TSK_EINVAL, "unknown state kind");
}

tsk_status krylov_schur(Operator* op, int m, int k, double tol, double delta, int pmax, int max_restarts,
                        const void* v0, uint64_t seed, double* mu_ri, double* lam_ri, double* resid, void* ritz,
                        tsk_ks_info* info) {
    if (!op) return fail(TSK_EINVAL, "null operator");
    if (op->is_complex()) return fail(TSK_EINVAL, "Krylov-Schur (real Schur form) needs a real operator");
    if (!op->ready()) return fail(TSK_ESTATE, "operator parameters or base flow not set");
    if (k < 1 || m < k + 2 || m > kMaxKrylov) return fail(TSK_EINVAL, "need 1 <= k and k + 2 <= m <= 96");
    if (int64_t(m) > op->n) return fail(TSK_EINVAL, "m exceeds the state dimension");
    if (pmax == 0) pmax = std::max(k, m / 2);
    if (pmax < k || pmax > m - 2) return fail(TSK_EINVAL, "need k <= p_max <= m - 2");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(TSK_EINVAL, "tol must be finite and >= 0");
    if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(TSK_EINVAL, "delta must be finite and >= 0");
    if (max_restarts < 0) return fail(TSK_EINVAL, "max_restarts must be >= 0");
    if (op->kind == StateKind::Real32)
        return krylov_schur_t<float>(op, m, k, tol, delta, pmax, max_restarts, v0, seed, mu_ri, lam_ri, resid, ritz,
                                     info);
    return krylov_schur_t<double>(op, m, k, tol, delta, pmax, max_restarts, v0, seed, mu_ri, lam_ri, resid, ritz,
                                  info);
}

}  // namespace tsk
