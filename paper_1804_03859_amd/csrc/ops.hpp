// Operator objects behind the opaque tsk_op handle, and the Arnoldi driver's
// device workspace.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace tsk {

// Device buffer owned by the library (hipMalloc/hipFree), grown on demand.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    tsk_status ensure(size_t want) {
        if (want <= bytes && ptr) return TSK_OK;
        release();
        if (want == 0) want = 16;
        if (hipMalloc(&ptr, want) != hipSuccess) {
            ptr = nullptr;
            return fail(TSK_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
        }
        bytes = want;
        return TSK_OK;
    }
    template <typename T> T* as() const { return static_cast<T*>(ptr); }
};

enum class StateKind { Complex64x2, Real64, Real32 };  // double2 / double / float

struct ArnoldiWork {
    // Ritz analyses of up to kSlots consecutive steps are in flight at once, in
    // batched launches on kAnaStreams side streams, each step with its own
    // eigensolver outputs (see arnoldi.hip).  An analysis at p ~ 50-60 takes
    // as long as ten to twenty-five steps, so fewer slots stall the operator
    // stream while it waits for a free one: with 16 instead of 24, 256^2 FP32
    // solves (62 steps) took 7.9-8.0 instead of 7.2-7.3 ms in interleaved runs;
    // 32 gained nothing more.
    static constexpr int kSlots = 24;
    // three analysis streams and the operator's stream use the 4 hardware queues a
    // process gets by default (GPU_MAX_HW_QUEUES); more streams would share a queue
    // and could put an analysis in front of a matvec
    static constexpr int kAnaStreams = 3;
    DevBuf V;         // (m+1) x n state vectors
    DevBuf H;         // (m+1) x m complex128, column-major
    DevBuf w;         // matvec output (state type)
    DevBuf w64;       // FP64 (or complex128) working copy during Gram-Schmidt
    DevBuf partial;   // per-block partial dot products
    DevBuf pnrm;      // per-block partial squared norms
    DevBuf h;         // reduced projection coefficients
    DevBuf scal;      // device scalars
    DevBuf eigS, eigMu, eigRes, sel;  // Hessenberg eigensolver, kSlots copies
    DevBuf eigY;      // unit Ritz coordinates of the wanted pairs (final step)
    DevBuf rr;        // RitzResult, kSlots copies
    DevBuf out;       // gathered outputs (mu, lambda, residual)
    DevBuf phys;      // physical field scratch (seeded start vector)
    DevBuf tmp;       // Lanczos on M^dagger M: the forward integration's output
    DevBuf V2;        // Krylov-Schur: second basis buffer (truncation writes here)
    DevBuf ksW;       // Krylov-Schur: m x p basis rotation (FP64)
    DevBuf ks_desc;   // batched restart phase: descriptor table of the restarting instances
    void* Vcur = nullptr;  // basis of the last run (V or V2)
    int m = 0, steps = 0;
    int64_t ldv = 0;
    // Owned by the first operator of a batch (the only one for a single run):
    DevBuf batch_desc;                 // kSlots KryDesc tables of the batch
    DevBuf batch_rr;                   // RitzResult of every instance and slot
    RitzResult* rr_host = nullptr;     // pinned copy of batch_rr
    int rr_host_count = 0;
    int* stop_host = nullptr;          // per-instance stop flags, coherent pinned memory read by the analyses
    int stop_count = 0;
    std::vector<hipEvent_t> ev_apply;  // 2 per matvec (start, end), timing
    hipEvent_t ev_cgs[kSlots] = {};    // basis vector j+1 and H column j ready (slot j % kSlots)
    hipEvent_t ev_eig[kSlots] = {};    // Ritz analysis of step j copied to the host
    hipStream_t side[kAnaStreams] = {};  // the process's analysis streams (shared, not owned; see arnoldi.hip)
    hipEvent_t ev_ana[kAnaStreams] = {};  // last analysis batch of each analysis stream done
    ~ArnoldiWork() {
        if (rr_host) (void)hipHostFree(rr_host);
        if (stop_host) (void)hipHostFree(stop_host);
        for (hipEvent_t e : ev_apply) (void)hipEventDestroy(e);
        for (int t = 0; t < kSlots; ++t) {
            if (ev_cgs[t]) (void)hipEventDestroy(ev_cgs[t]);
            if (ev_eig[t]) (void)hipEventDestroy(ev_eig[t]);
        }
        for (int a = 0; a < kAnaStreams; ++a)
            if (ev_ana[a]) (void)hipEventDestroy(ev_ana[a]);
    }
};

struct Operator {
    virtual ~Operator() = default;
    hipStream_t stream = nullptr;
    int64_t n = 0;           // state length in scalars (complex count if complex)
    StateKind kind = StateKind::Real64;
    double T = 0.0;
    bool params_set = false;
    bool base_set = false;
    // Stop-rule parameters of the wanted-set test (negative: the defaults of the
    // state type, kResFloorFp32 / kDupRelFp32 for FP32 states, 0 for FP64).
    double stop_res_floor = -1.0;
    double stop_dup_rel = -1.0;
    ArnoldiWork aw;

    bool is_complex() const { return kind == StateKind::Complex64x2; }
    int elem_bytes() const { return kind == StateKind::Real32 ? 4 : 8; }
    size_t state_bytes() const { return size_t(n) * (is_complex() ? 16 : size_t(elem_bytes())); }
    bool ready() const { return params_set && base_set; }

    virtual const char* name() const = 0;
    virtual tsk_status apply(const void* x, void* y) = 0;
    // y = M^dagger x, the transpose (conjugate transpose) of the discrete propagator
    // in the state's Euclidean inner product; operators without one fail.
    virtual tsk_status apply_adjoint(const void* /*x*/, void* /*y*/) {
        return fail(TSK_EINVAL, std::string("no adjoint propagator for ") + name());
    }
    virtual bool has_adjoint() const { return false; }
    virtual tsk_status from_physical(const void* phys, void* state) = 0;
    virtual tsk_status to_physical(const void* state, void* phys) = 0;
    // Number of reals in the physical field (complex fields count 2 per value).
    virtual int64_t physical_reals() const = 0;
};

// Factories (defined in cgle.hip / kolmo.hip).
tsk_status make_cgle(int n, double half_width, hipStream_t s, std::unique_ptr<Operator>* out);
tsk_status cgle_set_params(Operator* op, double U, double c_u, double c_d, double mu0, double mu2,
                           double dt, double T);
tsk_status make_kolmo(int N, tsk_precision prec, hipStream_t s, std::unique_ptr<Operator>* out);
tsk_status kolmo_set_params(Operator* op, double Re, double alpha, double dt, double T);
tsk_status kolmo_set_base_parallel(Operator* op, const double* U, const double* dOdy);
tsk_status kolmo_set_base_general(Operator* op, const double* U, const double* V, const double* Ox,
                                  const double* Oy);
bool is_kolmo(const Operator* op);
// Nonlinear forced equation on a Navier-Stokes operator (kolmo.hip): forcing that
// holds the laminar flow of wavenumber n_forcing steady, drift U0, optional extra
// forcing field (host N*N, nullable); steps of it; the packed laminar state; the
// general base flow set to a device state.
tsk_status kolmo_set_nonlinear(Operator* op, int n_forcing, double U0, const double* extra);
tsk_status kolmo_nonlinear_step(Operator* op, const void* x, void* y, int nsteps);  // 0: T/dt steps
tsk_status kolmo_laminar_state(Operator* op, void* x);
tsk_status kolmo_base_from_state(Operator* op, const void* x);
double kolmo_dt(const Operator* op);
int kolmo_nsteps(const Operator* op);
// Columns per wavefront of the column stepper: 0 = autotuned, 1 or 2 forced;
// get reports the forced or tuned value (0 = not tuned yet).
tsk_status kolmo_set_tuning(Operator* op, int cols);
tsk_status kolmo_get_tuning(const Operator* op, int* cols);
// Launch shape of the spectral-coupling stepper: wavefronts per workgroup, 0 =
// tuned (get: the shape of the last launch, 0 before the first).
tsk_status kolmo_set_stepper_waves(Operator* op, int w);
tsk_status kolmo_get_stepper_waves(const Operator* op, int* w);
// A Navier-Stokes operator whose base flow is parallel (column stepper; batchable).
bool kolmo_parallel(const Operator* op);
// The operator's own matvec runs the Bloch-sector stepper (colbloch.hpp).
bool kolmo_bloch(const Operator* op);
// The operator's own matvec runs the spectral-coupling stepper (colcouple.hpp).
bool kolmo_couple(const Operator* op);
// Largest kept wavenumber M = (N-1)/3 of a Navier-Stokes operator, -1 for others.
int kolmo_cutoff(const Operator* op);
bool is_cgle(const Operator* op);
// Resolvent mode of a Ginzburg-Landau operator: apply = R(omega) (forced
// integration over t_transient from rest), apply_adjoint = R(omega)^H;
// t_transient = 0 returns to the propagator.
tsk_status cgle_set_resolvent(Operator* op, double omega, double t_transient);

// Batched Navier-Stokes matvec of Arnoldi step j: x = V_j, y = w for every
// active instance of the descriptor table (kolmo.hip).
struct KryDesc;
struct KolmoBatch;
void kolmo_batch_free(KolmoBatch* b);
int kolmo_batch_groups(const KolmoBatch* b);  // grid-size groups of a batch plan
// The process's worker streams (one set per device, created on first use):
// the Arnoldi analyses, and the extra grid-size groups of a batched matvec.
tsk_status analysis_streams(hipStream_t (&out)[ArnoldiWork::kAnaStreams]);
struct KolmoBatchDeleter {
    void operator()(KolmoBatch* b) const { kolmo_batch_free(b); }
};
using KolmoBatchPtr = std::unique_ptr<KolmoBatch, KolmoBatchDeleter>;
tsk_status kolmo_batch_plan(Operator* const* ops, int count, const KryDesc* D_host, const KryDesc* D_dev,
                            KolmoBatchPtr* out);
tsk_status kolmo_batch_matvec(KolmoBatch* b, int j, hipStream_t s);
// Batched restart phase: instance i's matvec input becomes xbase[i] + j ldv, and
// steps j >= jmax[i] skip it.
tsk_status kolmo_batch_set_inputs(KolmoBatch* b, const void* const* xbase, const int* jmax, hipStream_t s);

// Ginzburg-Landau batches of one node count: the integrations of all instances
// (propagators or resolvents; with svd, the forward then the adjoint pass) in
// one launch per pass, one workgroup each.  The plan is left empty (per-instance
// launches) when the node counts differ.
struct CgleBatch;
void cgle_batch_free(CgleBatch* b);
struct CgleBatchDeleter {
    void operator()(CgleBatch* b) const { cgle_batch_free(b); }
};
using CgleBatchPtr = std::unique_ptr<CgleBatch, CgleBatchDeleter>;
tsk_status cgle_batch_plan(Operator* const* ops, int count, const KryDesc* D_host, bool svd, CgleBatchPtr* out);
tsk_status cgle_batch_matvec(CgleBatch* b, int j, hipStream_t s);

// Arnoldi driver (arnoldi.hip): `count` independent instances in lockstep.
// Per instance i: v0s[i] (nullable array / entry), seeds[i] (nullable array:
// seed i), outputs at mu_ri + 2k i, lam_ri + 2k i, resid + k i, ritz[i]
// (nullable array / entry), infos[i].  Returns the first negative status of a
// global failure; per-instance outcomes are in infos[i].status.
// svd = true: Lanczos on M^dagger M instead (every operator needs an adjoint);
// mu_ri then receives (sigma^2, 0).
// Batched restart phase (tsk_batch_krylov_schur): instances not converged at
// order m contract (Krylov-Schur, real states) and expand again in lockstep.
struct BatchRestart {
    double delta;      // wanted when |mu| >= 1 - delta
    int pmax;          // largest order kept
    int max_restarts;  // contractions per instance
    tsk_ks_info* infos;  // per instance (n_matvec, n_restarts, kept_last, ...)
};
tsk_status arnoldi_batch(Operator* const* ops, int count, int m, int k, double tol, const void* const* v0s,
                         const uint64_t* seeds, double* mu_ri, double* lam_ri, double* resid, void* const* ritz,
                         tsk_arnoldi_info* infos, bool svd = false, const BatchRestart* rs = nullptr);

// Krylov-Schur driver (arnoldi.hip): one real operator; arguments as tsk_krylov_schur.
tsk_status krylov_schur(Operator* op, int m, int k, double tol, double delta, int pmax, int max_restarts,
                        const void* v0, uint64_t seed, double* mu_ri, double* lam_ri, double* resid, void* ritz,
                        tsk_ks_info* info);
// The contraction on its own (hessenberg.hip); arguments as tsk_ks_contract.
tsk_status ks_contract_standalone(const double* H, int ldh, int m, double beta, int k, double delta, int pmax,
                                  void* mu, double* res, double* Hnew, double* W, int* kept, double* beta_new,
                                  hipStream_t s);

// Device Hessenberg eigensolver + wanted-set selection (hessenberg.hip), one
// wavefront per instance of the descriptor table (H, scal[2] = beta, scratch).
// full = true: accumulate all of Z and form every eigenvector (standalone use).
// real_h = true: H is real (real operators): real double-shift QR; with full,
// the standalone real solver (values and residuals only, beta from scal[2]).
struct KryDesc;
tsk_status hess_ritz_launch(const KryDesc* D, int count, int p, int k, double tol, bool full, hipStream_t s,
                            bool real_h = false, bool attrs_only = false);
// Several Krylov steps analysed by one launch (blockIdx.y = step, blockIdx.x =
// instance): step i reads the descriptor table tab[i] (its output slot) and its
// order p[i].  The Arnoldi driver gathers the steps whose Gram-Schmidt has
// finished into one launch, so the analyses of a backlog run side by side
// without a hardware queue each.
struct StepSet {
    static constexpr int kMax = 24;
    const KryDesc* tab[kMax];
    int p[kMax];
};
// The driver's analysis of n steps: tridiagonal (svd), real Hessenberg (real_h)
// or complex Hessenberg; no eigenvector accumulation.
tsk_status ritz_steps_launch(const StepSet& ss, int n, int count, int k, double tol, bool svd, bool real_h,
                             hipStream_t s);
// Lanczos Ritz analysis (symmetric tridiagonal T_p from H's diagonal and
// subdiagonal): as hess_ritz_launch, plus the unit Ritz coordinates of the
// wanted values in S[s*p + r].
tsk_status tridiag_ritz_launch(const KryDesc* D, int count, int p, int k, double tol, hipStream_t s);
tsk_status tridiag_ritz_launch_steps(const StepSet& ss, int n, int count, int pmax, int k, double tol,
                                     hipStream_t s);
// Krylov-Schur analysis and contraction of the order-m factorisations of the
// `count` instances D[0..count) (real H), one wavefront each: contract = 0
// analysis only, 1 unless the stop test is met, 2 always.  Results in D[i].rr
// (kept, beta), H and ksW.
tsk_status ks_contract_launch(const KryDesc* D, int m, int k, double tol, int contract, hipStream_t s,
                              int count = 1);
// Unit Ritz coordinates of the wanted pairs (inverse iteration on H_p): Y[s*p + r].
// Needs the attribute set by a prior hess_ritz_launch.
tsk_status ritz_coords_launch(const KryDesc* D, int count, int pmax, int k, hipStream_t s);  // p = steps

// FP32-state runs (the precision form).  The basis is rounded to FP32, so the
// Arnoldi relation, and with it the residual estimate, holds only to about
// u32 ||M||: a Ritz pair counts as converged once its estimate is below
// max(tol, kResFloorFp32 |mu|), kResFloorFp32 = 32 u32.  FP32 rounding also splits
// every multiple eigenvalue into a cluster; Ritz values closer than
// kDupRelFp32 |mu| (the stated FP32 eigenvalue accuracy, 2e-5) are copies of one
// eigenvalue.  FP64 runs use 0 for both (the rule of the Arnoldi stop test).
constexpr double kResFloorFp32 = 32.0 * 5.9604644775390625e-08;
constexpr double kDupRelFp32 = 2e-5;

// Fixed-point solvers (fixedpoint.hip) on the nonlinear equation of a
// Navier-Stokes operator; arguments as tsk_sfd, tsk_rpm, tsk_boostconv.
tsk_status fixed_point_sfd(Operator* op, void* x, double chi, double delta, int check_every, double tol,
                           int max_checks, double* hist, tsk_fp_info* info);
tsk_status fixed_point_rpm(Operator* op, void* x, int m, int k, double delta, double tol, int max_iter, double* hist,
                           tsk_fp_info* info);
tsk_status fixed_point_boostconv(Operator* op, void* x, int m, double tol, int max_iter, double* hist,
                                 tsk_fp_info* info);

// Learned start vector (mlp.hip): network object and entry points.
struct Mlp;
tsk_status mlp_create(int width, const double* lo, const double* hi, hipStream_t s, Mlp** out);
void mlp_free(Mlp* n);
int64_t mlp_param_count(const Mlp* n);
tsk_status mlp_init(Mlp* n, uint64_t seed);
tsk_status mlp_set_params(Mlp* n, const float* host);
tsk_status mlp_get_params(Mlp* n, float* host);
tsk_status mlp_forward(Mlp* n, const float* in, int B, float* out);
tsk_status mlp_gradients(Mlp* n, const float* in, const float* target, int B, float* grad, double* loss_host);
tsk_status mlp_train(Mlp* n, const float* in, const float* target, int B, int steps, double lr, double* loss_host);
tsk_status ritz_block_target(Operator* op, const void* ritz, int k, const int* use, float* target);
tsk_status mlp_start(Mlp* n, Operator* op, double Re, double alpha, double gamma, uint64_t seed, void* v0,
                     int* used);
// The standalone real Hessenberg eigensolver with its scratch in a fixed
// device array instead of per-call allocations (noalloc.hip); arguments as
// tsk_hessenberg_ritz_real_noalloc.
tsk_status hessenberg_ritz_real_noalloc(const double* H_dev, int ldh, int p, double beta, void* mu_dev,
                                        void* res_dev, hipStream_t s);

// Normal draws (rng.hip).
tsk_status normal_fill(double* out, int64_t count, uint64_t seed, hipStream_t s);
// out[i] = float(in[i]); out may alias the front of in.
tsk_status narrow_to_float(const double* in, float* out, int64_t count, hipStream_t s);

}  // namespace tsk
