// extern "C" entry points declared in include/tsk.h.  Every entry point catches
// C++ exceptions and turns them into a negative status; the message of the last
// failure on the calling thread is kept for tsk_last_error().
#include <cmath>
#include <cstring>
#include <vector>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "krylov.hpp"
#include "ops.hpp"

struct tsk_op_s {
    std::unique_ptr<tsk::Operator> op;
};

struct tsk_mlp_s {
    tsk::Mlp* net = nullptr;
    ~tsk_mlp_s() { tsk::mlp_free(net); }
};

namespace tsk {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

tsk_status fail(tsk_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

}  // namespace tsk

using namespace tsk;

#define TSK_GUARD(...)                                                                 \
    try {                                                                              \
        __VA_ARGS__                                                                    \
    } catch (const std::bad_alloc&) {                                                  \
        return fail(TSK_ENOMEM, "host allocation failed");                             \
    } catch (const std::exception& e) {                                                \
        return fail(TSK_EINVAL, std::string("internal error: ") + e.what());           \
    } catch (...) {                                                                    \
        return fail(TSK_EINVAL, "internal error");                                     \
    }

#define TSK_NEED(op)                                                                   \
    if (!(op) || !(op)->op) return fail(TSK_EINVAL, "null operator handle");

#define TSK_NEED_NET(h)                                                                \
    if (!(h) || !(h)->net) return fail(TSK_EINVAL, "null network handle");

extern "C" {

tsk_status tsk_create_cgle1d(tsk_op* out, int n, double half_width, void* hip_stream) {
    TSK_GUARD({
        if (!out) return fail(TSK_EINVAL, "null output handle");
        *out = nullptr;
        std::unique_ptr<Operator> op;
        TSK_TRY(make_cgle(n, half_width, static_cast<hipStream_t>(hip_stream), &op));
        auto* h = new tsk_op_s;
        h->op = std::move(op);
        *out = h;
        return TSK_OK;
    })
}

tsk_status tsk_set_params_cgle(tsk_op op, double U, double c_u, double c_d, double mu0, double mu2, double dt,
                               double T) {
    TSK_GUARD({
        TSK_NEED(op);
        return cgle_set_params(op->op.get(), U, c_u, c_d, mu0, mu2, dt, T);
    })
}

tsk_status tsk_create_kolmo2d(tsk_op* out, int N, tsk_precision precision, void* hip_stream) {
    TSK_GUARD({
        if (!out) return fail(TSK_EINVAL, "null output handle");
        *out = nullptr;
        std::unique_ptr<Operator> op;
        TSK_TRY(make_kolmo(N, precision, static_cast<hipStream_t>(hip_stream), &op));
        auto* h = new tsk_op_s;
        h->op = std::move(op);
        *out = h;
        return TSK_OK;
    })
}

tsk_status tsk_set_params_kolmo(tsk_op op, double Re, double alpha, double dt, double T) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_params(op->op.get(), Re, alpha, dt, T);
    })
}

tsk_status tsk_set_base_parallel(tsk_op op, const double* U_y, const double* dOmega_dy) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_base_parallel(op->op.get(), U_y, dOmega_dy);
    })
}

tsk_status tsk_set_base_kolmogorov(tsk_op op, int n_forcing) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!is_kolmo(op->op.get())) return fail(TSK_EINVAL, "not a Navier-Stokes operator");
        if (n_forcing < 1) return fail(TSK_EINVAL, "n_forcing must be >= 1");
        int64_t N = op->op->physical_reals();
        int n = 1;
        while (int64_t(n) * n < N) ++n;
        std::vector<double> U(n), dO(n);
        const double pi = 3.14159265358979323846264338327950288;
        for (int l = 0; l < n; ++l) {
            double y = 2.0 * pi * l / n;
            U[l] = std::sin(n_forcing * y);
            dO[l] = double(n_forcing) * n_forcing * U[l];
        }
        return kolmo_set_base_parallel(op->op.get(), U.data(), dO.data());
    })
}

tsk_status tsk_set_base_flow(tsk_op op, const double* U, const double* V, const double* dOmega_dx,
                             const double* dOmega_dy) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_base_general(op->op.get(), U, V, dOmega_dx, dOmega_dy);
    })
}

tsk_status tsk_set_tuning(tsk_op op, int columns_per_wave) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_tuning(op->op.get(), columns_per_wave);
    })
}

tsk_status tsk_get_tuning(tsk_op op, int* columns_per_wave) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!columns_per_wave) return fail(TSK_EINVAL, "null argument");
        return kolmo_get_tuning(op->op.get(), columns_per_wave);
    })
}

tsk_status tsk_set_stepper_waves(tsk_op op, int waves_per_group) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_stepper_waves(op->op.get(), waves_per_group);
    })
}

tsk_status tsk_get_stepper_waves(tsk_op op, int* waves_per_group) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!waves_per_group) return fail(TSK_EINVAL, "null argument");
        return kolmo_get_stepper_waves(op->op.get(), waves_per_group);
    })
}

tsk_status tsk_set_stop_rule(tsk_op op, double res_floor_rel, double dup_rel) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!std::isfinite(res_floor_rel) || !std::isfinite(dup_rel))
            return fail(TSK_EINVAL, "stop-rule parameters must be finite");
        if (res_floor_rel >= 1e-2 || dup_rel >= 1e-2)
            return fail(TSK_EINVAL, "stop-rule parameters must be below 1e-2");
        op->op->stop_res_floor = res_floor_rel < 0.0 ? -1.0 : res_floor_rel;
        op->op->stop_dup_rel = dup_rel < 0.0 ? -1.0 : dup_rel;
        return TSK_OK;
    })
}

tsk_status tsk_state_dim(tsk_op op, int64_t* n_scalars, int* is_complex, int* elem_bytes) {
    TSK_GUARD({
        TSK_NEED(op);
        if (n_scalars) *n_scalars = op->op->n;
        if (is_complex) *is_complex = op->op->is_complex() ? 1 : 0;
        if (elem_bytes) *elem_bytes = op->op->elem_bytes();
        return TSK_OK;
    })
}

tsk_status tsk_from_physical(tsk_op op, const void* phys_dev, void* state_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!phys_dev || !state_dev) return fail(TSK_EINVAL, "null buffer");
        return op->op->from_physical(phys_dev, state_dev);
    })
}

tsk_status tsk_to_physical(tsk_op op, const void* state_dev, void* phys_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!phys_dev || !state_dev) return fail(TSK_EINVAL, "null buffer");
        return op->op->to_physical(state_dev, phys_dev);
    })
}

tsk_status tsk_apply(tsk_op op, const void* x_dev, void* y_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!x_dev || !y_dev) return fail(TSK_EINVAL, "null buffer");
        if (x_dev == y_dev) return fail(TSK_EINVAL, "apply: input and output must not alias");
        return op->op->apply(x_dev, y_dev);
    })
}

tsk_status tsk_apply_adjoint(tsk_op op, const void* x_dev, void* y_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!x_dev || !y_dev) return fail(TSK_EINVAL, "null buffer");
        if (x_dev == y_dev) return fail(TSK_EINVAL, "apply_adjoint: input and output must not alias");
        return op->op->apply_adjoint(x_dev, y_dev);
    })
}

tsk_status tsk_set_resolvent(tsk_op op, double omega, double t_transient) {
    TSK_GUARD({
        TSK_NEED(op);
        return cgle_set_resolvent(op->op.get(), omega, t_transient);
    })
}

tsk_status tsk_optimal_perturbation(tsk_op op, int m, int k, double tol, const void* v0_dev, uint64_t seed,
                                    double* sigma, double* resid, void* vecs_dev, tsk_arnoldi_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        Operator* o = op->op.get();
        std::vector<double> mu(2 * size_t(std::max(k, 1)));
        const tsk_status st =
            arnoldi_batch(&o, 1, m, k, tol, &v0_dev, &seed, mu.data(), nullptr, resid, &vecs_dev, info, true);
        if (st < 0) return st;
        if (sigma)
            for (int q = 0; q < k; ++q) sigma[q] = std::sqrt(std::max(mu[2 * size_t(q)], 0.0));
        return st;
    })
}

tsk_status tsk_batch_optimal_perturbation(const tsk_op* ops, int count, int m, int k, double tol,
                                          const void* const* v0_devs, const uint64_t* seeds, double* sigma,
                                          double* resid, void* const* vecs_devs, tsk_arnoldi_info* infos) {
    TSK_GUARD({
        if (!ops || count < 1) return fail(TSK_EINVAL, "empty batch");
        std::vector<Operator*> o(count);
        for (int i = 0; i < count; ++i) {
            if (!ops[i] || !ops[i]->op) return fail(TSK_EINVAL, "null operator handle in batch");
            o[i] = ops[i]->op.get();
        }
        std::vector<double> mu(2 * size_t(count) * size_t(std::max(k, 1)));
        const tsk_status st = arnoldi_batch(o.data(), count, m, k, tol, v0_devs, seeds, mu.data(), nullptr, resid,
                                            vecs_devs, infos, true);
        if (st < 0) return st;
        if (sigma)
            for (size_t q = 0; q < size_t(count) * k; ++q) sigma[q] = std::sqrt(std::max(mu[2 * q], 0.0));
        return st;
    })
}

tsk_status tsk_set_nonlinear(tsk_op op, int n_forcing, double U0, const double* extra_forcing) {
    TSK_GUARD({
        TSK_NEED(op);
        return kolmo_set_nonlinear(op->op.get(), n_forcing, U0, extra_forcing);
    })
}

tsk_status tsk_laminar_state(tsk_op op, void* x_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!x_dev) return fail(TSK_EINVAL, "null buffer");
        return kolmo_laminar_state(op->op.get(), x_dev);
    })
}

tsk_status tsk_nonlinear_step(tsk_op op, const void* x_dev, void* y_dev, int nsteps) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!x_dev || !y_dev) return fail(TSK_EINVAL, "null buffer");
        if (x_dev == y_dev) return fail(TSK_EINVAL, "nonlinear_step: input and output must not alias");
        return kolmo_nonlinear_step(op->op.get(), x_dev, y_dev, nsteps);
    })
}

tsk_status tsk_set_base_from_state(tsk_op op, const void* x_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!x_dev) return fail(TSK_EINVAL, "null buffer");
        return kolmo_base_from_state(op->op.get(), x_dev);
    })
}

tsk_status tsk_sfd(tsk_op op, void* x_dev, double chi, double delta, int check_every, double tol, int max_checks,
                   double* hist, tsk_fp_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        return fixed_point_sfd(op->op.get(), x_dev, chi, delta, check_every, tol, max_checks, hist, info);
    })
}

tsk_status tsk_rpm(tsk_op op, void* x_dev, int m, int k, double delta, double tol, int max_iter, double* hist,
                   tsk_fp_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        return fixed_point_rpm(op->op.get(), x_dev, m, k, delta, tol, max_iter, hist, info);
    })
}

tsk_status tsk_boostconv(tsk_op op, void* x_dev, int m, double tol, int max_iter, double* hist, tsk_fp_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        return fixed_point_boostconv(op->op.get(), x_dev, m, tol, max_iter, hist, info);
    })
}

tsk_status tsk_arnoldi(tsk_op op, int m, int k, double tol, const void* v0_dev, uint64_t seed, double* mu_ri,
                       double* lambda_ri, double* resid, void* ritz_dev, tsk_arnoldi_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        Operator* o = op->op.get();
        return arnoldi_batch(&o, 1, m, k, tol, &v0_dev, &seed, mu_ri, lambda_ri, resid, &ritz_dev, info);
    })
}

tsk_status tsk_batch_arnoldi(const tsk_op* ops, int count, int m, int k, double tol, const void* const* v0_devs,
                             const uint64_t* seeds, double* mu_ri, double* lambda_ri, double* resid,
                             void* const* ritz_devs, tsk_arnoldi_info* infos) {
    TSK_GUARD({
        if (!ops || count < 1) return fail(TSK_EINVAL, "empty batch");
        std::vector<Operator*> o(count);
        for (int i = 0; i < count; ++i) {
            if (!ops[i] || !ops[i]->op) return fail(TSK_EINVAL, "null operator handle in batch");
            o[i] = ops[i]->op.get();
        }
        return arnoldi_batch(o.data(), count, m, k, tol, v0_devs, seeds, mu_ri, lambda_ri, resid, ritz_devs,
                             infos);
    })
}

tsk_status tsk_batch_krylov_schur(const tsk_op* ops, int count, int m, int k, double tol, double delta, int p_max,
                                  int max_restarts, const void* const* v0_devs, const uint64_t* seeds, double* mu_ri,
                                  double* lambda_ri, double* resid, void* const* ritz_devs, tsk_ks_info* infos) {
    TSK_GUARD({
        if (!ops || count < 1) return fail(TSK_EINVAL, "empty batch");
        std::vector<Operator*> o(count);
        for (int i = 0; i < count; ++i) {
            if (!ops[i] || !ops[i]->op) return fail(TSK_EINVAL, "null operator handle in batch");
            o[i] = ops[i]->op.get();
            if (o[i]->is_complex()) return fail(TSK_EINVAL, "Krylov-Schur (real Schur form) needs real operators");
        }
        if (k < 1 || m < k + 2 || m > kMaxKrylov) return fail(TSK_EINVAL, "need 1 <= k and k + 2 <= m <= 96");
        if (p_max == 0) p_max = std::max(k, m / 2);
        if (p_max < k || p_max > m - 2) return fail(TSK_EINVAL, "need k <= p_max <= m - 2");
        if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(TSK_EINVAL, "delta must be finite and >= 0");
        if (max_restarts < 0) return fail(TSK_EINVAL, "max_restarts must be >= 0");
        BatchRestart rs{delta, p_max, max_restarts, infos};
        return arnoldi_batch(o.data(), count, m, k, tol, v0_devs, seeds, mu_ri, lambda_ri, resid, ritz_devs, nullptr,
                             false, &rs);
    })
}

tsk_status tsk_krylov_schur(tsk_op op, int m, int k, double tol, double delta, int p_max, int max_restarts,
                            const void* v0_dev, uint64_t seed, double* mu_ri, double* lambda_ri, double* resid,
                            void* ritz_dev, tsk_ks_info* info) {
    TSK_GUARD({
        TSK_NEED(op);
        return krylov_schur(op->op.get(), m, k, tol, delta, p_max, max_restarts, v0_dev, seed, mu_ri, lambda_ri,
                            resid, ritz_dev, info);
    })
}

tsk_status tsk_ks_contract(const double* H_dev, int ldh, int m, double beta, int k, double delta, int p_max,
                           void* mu_dev, double* res_dev, double* Hnew_dev, double* W_dev, int* kept,
                           double* beta_new, void* hip_stream) {
    TSK_GUARD({
        if (!H_dev || !mu_dev || !res_dev || !Hnew_dev || !W_dev || !kept || !beta_new)
            return fail(TSK_EINVAL, "null buffer");
        if (k < 1 || m < k + 2 || m > kMaxKrylov || ldh < m)
            return fail(TSK_EINVAL, "need 1 <= k, k + 2 <= m <= 96 and ldh >= m");
        if (p_max == 0) p_max = std::max(k, m / 2);
        if (p_max < k || p_max > m - 2) return fail(TSK_EINVAL, "need k <= p_max <= m - 2");
        if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(TSK_EINVAL, "delta must be finite and >= 0");
        return ks_contract_standalone(H_dev, ldh, m, beta, k, delta, p_max, mu_dev, res_dev, Hnew_dev, W_dev, kept,
                                      beta_new, static_cast<hipStream_t>(hip_stream));
    })
}

tsk_status tsk_last_hessenberg(tsk_op op, double* H_host, int* m_out, int* steps_out) {
    TSK_GUARD({
        TSK_NEED(op);
        ArnoldiWork& W = op->op->aw;
        if (!W.H.ptr || W.m == 0) return fail(TSK_ESTATE, "no Arnoldi run on this operator");
        if (m_out) *m_out = W.m;
        if (steps_out) *steps_out = W.steps;
        if (H_host) {
            TSK_HIP(hipStreamSynchronize(op->op->stream));
            TSK_HIP(hipMemcpy(H_host, W.H.ptr, size_t(W.m + 1) * W.m * sizeof(double2), hipMemcpyDeviceToHost));
        }
        return TSK_OK;
    })
}

tsk_status tsk_last_basis(tsk_op op, const void** V_dev, int64_t* ld) {
    TSK_GUARD({
        TSK_NEED(op);
        ArnoldiWork& W = op->op->aw;
        if (!W.V.ptr || W.m == 0) return fail(TSK_ESTATE, "no Arnoldi run on this operator");
        if (V_dev) *V_dev = W.Vcur ? W.Vcur : W.V.ptr;
        if (ld) *ld = W.ldv;
        return TSK_OK;
    })
}

tsk_status tsk_hessenberg_ritz(const void* H_dev, int ldh, int p, double beta, void* mu_dev, void* Y_dev,
                               void* res_dev, void* hip_stream) {
    TSK_GUARD({
        if (!H_dev || !mu_dev || !Y_dev || !res_dev) return fail(TSK_EINVAL, "null buffer");
        if (p < 1 || p > kMaxKrylov || ldh < p) return fail(TSK_EINVAL, "need 1 <= p <= 96 and ldh >= p");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        DevBuf Z, S, rr, scal, dd;
        TSK_TRY(Z.ensure(size_t(p) * p * sizeof(double2)));
        TSK_TRY(S.ensure(size_t(p) * p * sizeof(double2)));
        TSK_TRY(rr.ensure(sizeof(RitzResult)));
        TSK_TRY(scal.ensure(64 * sizeof(double)));
        TSK_TRY(dd.ensure(sizeof(KryDesc)));
        double sc[64] = {0};
        sc[2] = beta;
        RitzResult r0{};
        KryDesc d;
        std::memset(&d, 0, sizeof(d));
        d.H = const_cast<double2*>(static_cast<const double2*>(H_dev));
        d.ldh = ldh;
        d.scal = scal.as<double>();
        d.Z = Z.as<double2>();
        d.S = S.as<double2>();
        d.Y = static_cast<double2*>(Y_dev);
        d.mu = static_cast<double2*>(mu_dev);
        d.res = static_cast<double*>(res_dev);
        d.rr = rr.as<RitzResult>();
        d.active = 1;
        TSK_HIP(hipMemcpyAsync(scal.ptr, sc, sizeof(sc), hipMemcpyHostToDevice, s));
        TSK_HIP(hipMemcpyAsync(rr.ptr, &r0, sizeof(r0), hipMemcpyHostToDevice, s));
        TSK_HIP(hipMemcpyAsync(dd.ptr, &d, sizeof(d), hipMemcpyHostToDevice, s));
        TSK_TRY(hess_ritz_launch(dd.as<KryDesc>(), 1, p, 0, 0.0, true, s));
        RitzResult h{};
        TSK_HIP(hipMemcpyAsync(&h, rr.ptr, sizeof(RitzResult), hipMemcpyDeviceToHost, s));
        TSK_HIP(hipStreamSynchronize(s));
        if (h.nonfinite) return fail(TSK_ENONFINITE, "H or beta is not finite");
        if (h.eig_fail) return fail(TSK_EEIG, "Hessenberg QR did not converge");
        return TSK_OK;
    })
}

tsk_status tsk_hessenberg_ritz_real(const double* H_dev, int ldh, int p, double beta, void* mu_dev, void* res_dev,
                                    void* hip_stream) {
    TSK_GUARD({
        if (!H_dev || !mu_dev || !res_dev) return fail(TSK_EINVAL, "null buffer");
        if (p < 1 || p > kMaxKrylov || ldh < p) return fail(TSK_EINVAL, "need 1 <= p <= 96 and ldh >= p");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        DevBuf Hc, S, rr, scal, dd;
        const size_t ne = size_t(ldh) * p;
        TSK_TRY(Hc.ensure(ne * sizeof(double2)));
        TSK_TRY(S.ensure(size_t(p) * p * sizeof(double2)));
        TSK_TRY(rr.ensure(sizeof(RitzResult)));
        TSK_TRY(scal.ensure(64 * sizeof(double)));
        TSK_TRY(dd.ensure(sizeof(KryDesc)));
        // real values into the real parts of a complex copy (the layout the solver reads)
        TSK_HIP(hipMemsetAsync(Hc.ptr, 0, ne * sizeof(double2), s));
        TSK_HIP(hipMemcpy2DAsync(Hc.ptr, sizeof(double2), H_dev, sizeof(double), sizeof(double), ne,
                                 hipMemcpyDeviceToDevice, s));
        double sc[64] = {0};
        sc[2] = beta;
        RitzResult r0{};
        KryDesc d;
        std::memset(&d, 0, sizeof(d));
        d.H = Hc.as<double2>();
        d.ldh = ldh;
        d.scal = scal.as<double>();
        d.S = S.as<double2>();
        d.mu = static_cast<double2*>(mu_dev);
        d.res = static_cast<double*>(res_dev);
        d.rr = rr.as<RitzResult>();
        d.active = 1;
        TSK_HIP(hipMemcpyAsync(scal.ptr, sc, sizeof(sc), hipMemcpyHostToDevice, s));
        TSK_HIP(hipMemcpyAsync(rr.ptr, &r0, sizeof(r0), hipMemcpyHostToDevice, s));
        TSK_HIP(hipMemcpyAsync(dd.ptr, &d, sizeof(d), hipMemcpyHostToDevice, s));
        TSK_TRY(hess_ritz_launch(dd.as<KryDesc>(), 1, p, 0, 0.0, true, s, true));
        RitzResult h{};
        TSK_HIP(hipMemcpyAsync(&h, rr.ptr, sizeof(RitzResult), hipMemcpyDeviceToHost, s));
        TSK_HIP(hipStreamSynchronize(s));
        if (h.nonfinite) return fail(TSK_ENONFINITE, "H or beta is not finite");
        if (h.eig_fail) return fail(TSK_EEIG, "Hessenberg QR did not converge");
        return TSK_OK;
    })
}

tsk_status tsk_hessenberg_ritz_real_noalloc(const double* H_dev, int ldh, int p, double beta, void* mu_dev,
                                            void* res_dev, void* hip_stream) {
    TSK_GUARD({
        return hessenberg_ritz_real_noalloc(H_dev, ldh, p, beta, mu_dev, res_dev,
                                            static_cast<hipStream_t>(hip_stream));
    })
}

tsk_status tsk_normal_fill(double* out_dev, int64_t count, uint64_t seed, void* hip_stream) {
    TSK_GUARD({
        if (!out_dev || count < 0) return fail(TSK_EINVAL, "bad output buffer or count");
        return normal_fill(out_dev, count, seed, static_cast<hipStream_t>(hip_stream));
    })
}

tsk_status tsk_mlp_create(tsk_mlp* out, int width, const double* in_lo, const double* in_hi, void* hip_stream) {
    TSK_GUARD({
        if (!out || !in_lo || !in_hi) return fail(TSK_EINVAL, "null argument");
        *out = nullptr;
        Mlp* n = nullptr;
        TSK_TRY(mlp_create(width, in_lo, in_hi, static_cast<hipStream_t>(hip_stream), &n));
        auto* h = new tsk_mlp_s;
        h->net = n;
        *out = h;
        return TSK_OK;
    })
}

tsk_status tsk_mlp_param_count(tsk_mlp net, int64_t* count) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!count) return fail(TSK_EINVAL, "null argument");
        *count = mlp_param_count(net->net);
        return TSK_OK;
    })
}

tsk_status tsk_mlp_init(tsk_mlp net, uint64_t seed) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        return mlp_init(net->net, seed);
    })
}

tsk_status tsk_mlp_set_params(tsk_mlp net, const float* params_host) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!params_host) return fail(TSK_EINVAL, "null parameter array");
        return mlp_set_params(net->net, params_host);
    })
}

tsk_status tsk_mlp_get_params(tsk_mlp net, float* params_host) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!params_host) return fail(TSK_EINVAL, "null parameter array");
        return mlp_get_params(net->net, params_host);
    })
}

tsk_status tsk_mlp_forward(tsk_mlp net, const float* in_dev, int batch, float* out_dev) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!in_dev || !out_dev) return fail(TSK_EINVAL, "null buffer");
        return mlp_forward(net->net, in_dev, batch, out_dev);
    })
}

tsk_status tsk_mlp_gradients(tsk_mlp net, const float* in_dev, const float* target_dev, int batch, float* grad_dev,
                             double* loss_host) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!in_dev || !target_dev) return fail(TSK_EINVAL, "null buffer");
        return mlp_gradients(net->net, in_dev, target_dev, batch, grad_dev, loss_host);
    })
}

tsk_status tsk_mlp_train(tsk_mlp net, const float* in_dev, const float* target_dev, int batch, int steps, double lr,
                         double* loss_host) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        if (!in_dev || !target_dev) return fail(TSK_EINVAL, "null buffer");
        return mlp_train(net->net, in_dev, target_dev, batch, steps, lr, loss_host);
    })
}

tsk_status tsk_ritz_block_target(tsk_op op, const void* ritz_dev, int k, const int* use_host, float* target_dev) {
    TSK_GUARD({
        TSK_NEED(op);
        if (!ritz_dev || !target_dev) return fail(TSK_EINVAL, "null buffer");
        return ritz_block_target(op->op.get(), ritz_dev, k, use_host, target_dev);
    })
}

tsk_status tsk_mlp_start(tsk_mlp net, tsk_op op, double Re, double alpha, double gamma, uint64_t seed, void* v0_dev,
                         int* used_net) {
    TSK_GUARD({
        TSK_NEED_NET(net);
        TSK_NEED(op);
        if (!v0_dev) return fail(TSK_EINVAL, "null start-vector buffer");
        return mlp_start(net->net, op->op.get(), Re, alpha, gamma, seed, v0_dev, used_net);
    })
}

void tsk_mlp_destroy(tsk_mlp net) {
    try {
        delete net;
    } catch (...) {
    }
}

void tsk_destroy(tsk_op op) {
    try {
        if (op) {
            if (op->op) (void)hipStreamSynchronize(op->op->stream);
            delete op;
        }
    } catch (...) {
    }
}

const char* tsk_status_str(int status) {
    switch (status) {
        case TSK_OK: return "converged";
        case TSK_NOT_CONVERGED: return "not converged after m matvecs";
        case TSK_BREAKDOWN: return "Arnoldi breakdown (invariant subspace)";
        case TSK_EINVAL: return "invalid argument";
        case TSK_ENOMEM: return "out of memory";
        case TSK_EHIP: return "HIP runtime error";
        case TSK_ENONFINITE: return "non-finite value";
        case TSK_ESTATE: return "call out of order";
        case TSK_EEIG: return "Hessenberg QR did not converge";
        default: return "unknown status";
    }
}

const char* tsk_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
