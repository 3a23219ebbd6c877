// Linear complex Ginzburg-Landau operator and its Crank-Nicolson time stepper.
//
// Equation (Sec. 2.3.2, eq. "ginzburg-landau equation"):
//     du/dt = -nu u_x + gamma u_xx + mu(x) u,  mu(x) = mu0 - c_u^2 + mu2 x^2 / 2,
// with nu = U + 2 i c_u and gamma = 1 + i c_d.  Second-order central
// differences on n interior nodes (Dirichlet ends) give the tridiagonal L_h;
// one matvec of M = exp(L T) is T/dt Crank-Nicolson steps
//     (I - dt/2 L_h) u+ = (I + dt/2 L_h) u.
//
// Kernel design: the whole state (n <= 1024 complex128, 16 KB) stays in one
// workgroup for the full integration, one thread per node.  The implicit solve
// is parallel cyclic reduction (Hockney & Jesshope): level l eliminates the
// couplings at distance 2^l, so after ceil(log2 n) levels every equation is
// decoupled.  The elimination multipliers of the constant matrix are computed
// once on the host when the parameters are set, so a time step is the
// three-point right-hand side plus, per level, two neighbour reads from LDS and
// two complex multiply-adds per node.  The matrix is strictly diagonally
// dominant, so no pivoting is needed.
#include <complex>
#include <vector>

#include "krylov.hpp"
#include "ops.hpp"

namespace tsk {

namespace {

constexpr int kCgleMaxN = 1024;
constexpr int kCgleMaxLevels = 10;

// One Crank-Nicolson integration (one workgroup).  Propagator: nsteps steps of
// the state in.  Forced (the resolvent mode): in is the forcing f^ of
// u' = L u + f^ e^{i omega t}; the run starts from rest, the forcing enters by
// the trapezoidal rule (dt/2 (f_n + f_{n+1}) = c1 e^{i omega t_n} f^ with
// c1 = dt/2 (1 + e^{i omega dt})), and the output is the phase-normalised state
// u(t_N) e^{-i omega t_N}.
struct CnJob {
    const double2* in;    // input of Krylov step j: in + j * in_stride
    long long in_stride;  // elements (0: one fixed input)
    double2* out;
    const double2* tab;   // rhs_main[n] | alpha[levels n] | gamma[levels n] | binv[n]
    double2 rsub, rsup;   // dt/2 times the constant sub/super diagonals
    double2 c1;
    double omega, dt;
    int n, levels, nsteps, forced;
};

// LV = the number of reduction levels, ceil(log2 n): a compile-time count keeps
// the per-level multipliers in registers.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <int LV>
__device__ __forceinline__ void cn_integrate(const CnJob& jb, int j) {
    __shared__ double2 bufA[kCgleMaxN];
    __shared__ double2 bufB[kCgleMaxN];
    constexpr int levels = LV;
    const int n = jb.n;
    const int i = threadIdx.x;
    const bool act = i < n;
    const double2 zero = cmk<double2>(0.0, 0.0);
    const double2* __restrict__ alpha = jb.tab + n;
    const double2* __restrict__ gamma = alpha + size_t(levels) * n;
    double2 al[LV], ga[LV];
#pragma unroll
    for (int l = 0; l < LV; ++l) {
        al[l] = act ? alpha[l * n + i] : zero;
        ga[l] = act ? gamma[l * n + i] : zero;
    }
    const double2 rm = act ? jb.tab[i] : zero;
    const double2 bi = act ? gamma[size_t(levels) * n + i] : zero;
    const double2* __restrict__ uin = jb.in + j * jb.in_stride;
    const bool forced = jb.forced != 0;
    const double2 fh = (forced && act) ? cmul(jb.c1, uin[i]) : zero;
    double2 u = (!forced && act) ? uin[i] : zero;
    // forcing phases e^{i omega dt s}: lane l of every wave evaluates step s0 + l
    // once per 64 steps, step s reads lane s - s0
    const int lane = i & (kWave - 1);
    double2 ph = zero;
    for (int st = 0; st < jb.nsteps; ++st) {
        // explicit half: d = (I + dt/2 L) u (+ the forcing)
        bufA[i] = u;
        __syncthreads();
        double2 um = (i > 0 && act) ? bufA[i - 1] : zero;
        double2 up = (i + 1 < n) ? bufA[i + 1] : zero;
        double2 d = cadd(cmul(rm, u), cadd(cmul(jb.rsub, um), cmul(jb.rsup, up)));
        if (forced) {
            if ((st & (kWave - 1)) == 0) {
                double sn, cs;
                sincos(jb.omega * jb.dt * double(st + lane), &sn, &cs);
                ph = cmk<double2>(cs, sn);
            }
            const int sl = st & (kWave - 1);  // uniform, < 64
            const double2 e = cmk<double2>(lane_bcast(ph.x, sl), lane_bcast(ph.y, sl));
            d = cadd(d, cmul(e, fh));
        }
        // implicit half by cyclic reduction, ping-pong between two LDS buffers
        double2* src = bufA;  // level 0 swaps to bufB: bufA is still being read for the stencil
        double2* dst = bufB;
        int s = 1;
#pragma unroll
        for (int l = 0; l < LV; ++l) {
            double2* t = src; src = dst; dst = t;  // write into the buffer read last level
            src[i] = d;
            __syncthreads();
            // out-of-range neighbours have zero multipliers: clamp the index
            // instead of branching (the state is finite, so 0 * x = 0 exactly)
            const double2 dm = src[max(i - s, 0)];
            const double2 dp = src[min(i + s, n - 1)];
            d = cadd(d, cadd(cmul(al[l], dm), cmul(ga[l], dp)));
            s <<= 1;
        }
        u = cmul(d, bi);
        __syncthreads();
    }
    if (forced) {
        double sn, cs;
        sincos(jb.omega * jb.dt * double(jb.nsteps), &sn, &cs);
        u = cmul(u, cmk<double2>(cs, -sn));
    }
    if (act) jb.out[i] = u;
}

// n <= 2^LV nodes, one thread each, rounded up to whole wavefronts: the bound
// leaves up to 256 registers per lane for LV <= 9.
constexpr int cn_threads_max(int lv) { return (1 << lv) < kWave ? kWave : (1 << lv); }

template <int LV>
__global__ __launch_bounds__(cn_threads_max(LV)) void k_cgle_cn(CnJob jb) { cn_integrate<LV>(jb, 0); }

// A batch of integrations (one per workgroup), Krylov step j of each.
template <int LV>
__global__ __launch_bounds__(cn_threads_max(LV)) void k_cgle_cn_batch(const CnJob* __restrict__ jobs, int j) {
    const CnJob jb = jobs[blockIdx.x];
    cn_integrate<LV>(jb, j);
}

// Launch with the level count as a template argument (jobs == null: the single
// job `one`).
template <int LV>
void launch_cn(const CnJob& one, const CnJob* jobs, int count, int j, int threads, hipStream_t s) {
    static_assert(cn_threads_max(LV) <= kCgleMaxN, "reduction depth beyond the node limit");
    if (jobs)
        hipLaunchKernelGGL(k_cgle_cn_batch<LV>, dim3(count), dim3(threads), 0, s, jobs, j);
    else
        hipLaunchKernelGGL(k_cgle_cn<LV>, dim3(1), dim3(threads), 0, s, one);
}

tsk_status launch_cn_levels(int levels, const CnJob& one, const CnJob* jobs, int count, int j, int threads,
                            hipStream_t s) {
    if (levels < 1 || levels > 10 || threads > cn_threads_max(levels) || threads % kWave)
        return fail(TSK_EINVAL, "CGLE launch shape does not fit the reduction depth");
    switch (levels) {
        case 1: launch_cn<1>(one, jobs, count, j, threads, s); break;
        case 2: launch_cn<2>(one, jobs, count, j, threads, s); break;
        case 3: launch_cn<3>(one, jobs, count, j, threads, s); break;
        case 4: launch_cn<4>(one, jobs, count, j, threads, s); break;
        case 5: launch_cn<5>(one, jobs, count, j, threads, s); break;
        case 6: launch_cn<6>(one, jobs, count, j, threads, s); break;
        case 7: launch_cn<7>(one, jobs, count, j, threads, s); break;
        case 8: launch_cn<8>(one, jobs, count, j, threads, s); break;
        case 9: launch_cn<9>(one, jobs, count, j, threads, s); break;
        case 10: launch_cn<10>(one, jobs, count, j, threads, s); break;
        default: return fail(TSK_EINVAL, "CGLE reduction depth out of range");
    }
    TSK_HIP(hipGetLastError());
    return TSK_OK;
}

// Tables of one Crank-Nicolson propagator: the explicit stencil (main diagonal
// per node, constant sub/super coefficients) and the cyclic-reduction
// multipliers of the implicit matrix.
struct CnTables {
    double2 rsub{}, rsup{};
    DevBuf tab;  // rhs_main[n] | alpha[levels*n] | gamma[levels*n] | binv[n]
};

struct CgleOp final : Operator {
    int nn = 0;
    double half_width = 0.0;
    int levels = 0, nsteps = 0;
    double dt = 0.0;
    CnTables fwd, adj;  // L_h and its conjugate transpose (the adjoint propagator)
    // resolvent mode: apply = R(omega) by ntrans forced steps from rest
    bool resolvent = false;
    double omega = 0.0, ttrans = 0.0;
    int ntrans = 0;

    const char* name() const override { return "cgle1d"; }
    int64_t physical_reals() const override { return 2 * int64_t(nn); }

    tsk_status set_params(double U, double c_u, double c_d, double mu0, double mu2, double dt, double TT) {
        using cd = std::complex<double>;
        if (!(dt > 0.0) || !(TT > 0.0) || !std::isfinite(dt) || !std::isfinite(TT))
            return fail(TSK_EINVAL, "dt and T must be positive and finite");
        double ns = TT / dt;
        int nsi = int(std::lround(ns));
        if (nsi < 1 || std::fabs(ns - nsi) > 1e-9 * std::max(1.0, ns))
            return fail(TSK_EINVAL, "T must be an integer multiple of dt");
        const int n_ = nn;
        const double dx = 2.0 * half_width / (n_ + 1);
        const cd nu(U, 2.0 * c_u), gam(1.0, c_d);
        const cd sub = gam / (dx * dx) + nu / (2.0 * dx);
        const cd sup = gam / (dx * dx) - nu / (2.0 * dx);
        std::vector<cd> mainv(n_), mainh(n_);
        for (int j = 0; j < n_; ++j) {
            double x = -half_width + dx * (j + 1);
            double mux = (mu0 - c_u * c_u) + mu2 * x * x / 2.0;
            mainv[j] = -2.0 * gam / (dx * dx) + mux;
            mainh[j] = std::conj(mainv[j]);
        }
        int L = 0;
        while ((1 << L) < n_) ++L;
        // L_h^H: conjugated main diagonal, sub and super diagonals swapped and conjugated
        TSK_TRY(build(fwd, sub, sup, mainv, 0.5 * dt, L));
        TSK_TRY(build(adj, std::conj(sup), std::conj(sub), mainh, 0.5 * dt, L));
        levels = L;
        nsteps = nsi;
        T = TT;
        this->dt = dt;
        if (resolvent) ntrans = std::max(1, int(std::lround(ttrans / dt)));
        params_set = true;
        return TSK_OK;
    }

    // Crank-Nicolson tables of the tridiagonal (sub, mainv, sup), h = dt/2.
    tsk_status build(CnTables& tb, std::complex<double> sub, std::complex<double> sup,
                     const std::vector<std::complex<double>>& mainv, double h, int L) {
        using cd = std::complex<double>;
        const int n_ = nn;
        std::vector<cd> a(n_), b(n_), c(n_);
        for (int j = 0; j < n_; ++j) {
            a[j] = j > 0 ? -h * sub : cd(0.0);
            b[j] = 1.0 - h * mainv[j];
            c[j] = j + 1 < n_ ? -h * sup : cd(0.0);
        }
        std::vector<cd> al(size_t(L) * n_), ga(size_t(L) * n_);
        for (int l = 0, s = 1; l < L; ++l, s <<= 1) {
            std::vector<cd> a2(n_), b2(n_), c2(n_);
            for (int j = 0; j < n_; ++j) {
                cd alpha = j - s >= 0 ? -a[j] / b[j - s] : cd(0.0);
                cd gamma = j + s < n_ ? -c[j] / b[j + s] : cd(0.0);
                al[size_t(l) * n_ + j] = alpha;
                ga[size_t(l) * n_ + j] = gamma;
                a2[j] = j - s >= 0 ? alpha * a[j - s] : cd(0.0);
                c2[j] = j + s < n_ ? gamma * c[j + s] : cd(0.0);
                b2[j] = b[j] + (j - s >= 0 ? alpha * c[j - s] : cd(0.0)) + (j + s < n_ ? gamma * a[j + s] : cd(0.0));
            }
            a.swap(a2); b.swap(b2); c.swap(c2);
        }
        std::vector<double2> host(size_t(n_) * (2 + 2 * L));
        size_t o = 0;
        for (int j = 0; j < n_; ++j) { cd r = 1.0 + h * mainv[j]; host[o++] = cmk<double2>(r.real(), r.imag()); }
        for (const cd& v : al) host[o++] = cmk<double2>(v.real(), v.imag());
        for (const cd& v : ga) host[o++] = cmk<double2>(v.real(), v.imag());
        for (int j = 0; j < n_; ++j) { cd r = 1.0 / b[j]; host[o++] = cmk<double2>(r.real(), r.imag()); }
        TSK_TRY(tb.tab.ensure(host.size() * sizeof(double2)));
        TSK_HIP(hipMemcpy(tb.tab.ptr, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice));
        cd rs = h * sub, rp = h * sup;
        tb.rsub = cmk<double2>(rs.real(), rs.imag());
        tb.rsup = cmk<double2>(rp.real(), rp.imag());
        return TSK_OK;
    }

    // Propagator (forced = false: T/dt steps of x) or resolvent (forced = true:
    // x is the forcing, ntrans steps at frequency w from rest).
    CnJob job(const CnTables& tb, bool forced, double w) const {
        CnJob jb{};
        jb.tab = tb.tab.as<double2>();
        jb.rsub = tb.rsub;
        jb.rsup = tb.rsup;
        jb.n = nn;
        jb.levels = levels;
        jb.dt = dt;
        jb.forced = forced ? 1 : 0;
        if (forced) {
            const double h = 0.5 * dt;
            jb.c1 = cmk<double2>(h * (1.0 + std::cos(w * dt)), h * std::sin(w * dt));
            jb.omega = w;
            jb.nsteps = ntrans;
        } else {
            jb.nsteps = nsteps;
        }
        return jb;
    }
    int threads() const { return (nn + kWave - 1) / kWave * kWave; }
    tsk_status run(const CnTables& tb, const void* x, void* y, bool forced, double w) {
        if (!ready()) return fail(TSK_ESTATE, "CGLE parameters not set");
        if (x == y) return fail(TSK_EINVAL, "input and output must not alias");
        CnJob jb = job(tb, forced, w);
        jb.in = static_cast<const double2*>(x);
        jb.out = static_cast<double2*>(y);
        return launch_cn_levels(levels, jb, nullptr, 1, 0, threads(), stream);
    }
    tsk_status apply(const void* x, void* y) override { return run(fwd, x, y, resolvent, omega); }
    // M^H: Crank-Nicolson with L_h^H (the two factors of a step commute, so this is
    // the conjugate transpose of the forward propagator).  Resolvent mode:
    // R(omega)^H = the forced integration with L_h^H at frequency -omega.
    tsk_status apply_adjoint(const void* x, void* y) override { return run(adj, x, y, resolvent, -omega); }
    bool has_adjoint() const override { return true; }
    tsk_status from_physical(const void* phys, void* state) override {
        TSK_HIP(hipMemcpyAsync(state, phys, state_bytes(), hipMemcpyDeviceToDevice, stream));
        return TSK_OK;
    }
    tsk_status to_physical(const void* state, void* phys) override {
        TSK_HIP(hipMemcpyAsync(phys, state, state_bytes(), hipMemcpyDeviceToDevice, stream));
        return TSK_OK;
    }
};

}  // namespace

tsk_status make_cgle(int n, double half_width, hipStream_t s, std::unique_ptr<Operator>* out) {
    if (n < 2 || n > kCgleMaxN) return fail(TSK_EINVAL, "CGLE node count must be in [2, 1024]");
    if (!(half_width > 0.0) || !std::isfinite(half_width)) return fail(TSK_EINVAL, "half_width must be positive");
    auto op = std::make_unique<CgleOp>();
    op->nn = n;
    op->half_width = half_width;
    op->n = n;
    op->kind = StateKind::Complex64x2;
    op->stream = s;
    op->base_set = true;  // the CGLE has no base flow
    *out = std::move(op);
    return TSK_OK;
}

tsk_status cgle_set_params(Operator* op, double U, double c_u, double c_d, double mu0, double mu2, double dt,
                           double T) {
    auto* c = dynamic_cast<CgleOp*>(op);
    if (!c) return fail(TSK_EINVAL, "not a Ginzburg-Landau operator");
    return c->set_params(U, c_u, c_d, mu0, mu2, dt, T);
}

bool is_cgle(const Operator* op) { return dynamic_cast<const CgleOp*>(op) != nullptr; }

tsk_status cgle_set_resolvent(Operator* op, double omega, double t_transient) {
    auto* c = dynamic_cast<CgleOp*>(op);
    if (!c) return fail(TSK_EINVAL, "the resolvent mode needs a Ginzburg-Landau operator (complex state)");
    if (!c->params_set) return fail(TSK_ESTATE, "CGLE parameters not set");
    if (!std::isfinite(omega) || !std::isfinite(t_transient) || t_transient < 0.0)
        return fail(TSK_EINVAL, "omega must be finite and t_transient >= 0");
    if (t_transient == 0.0) {
        c->resolvent = false;
        return TSK_OK;
    }
    const double steps = t_transient / c->dt;
    if (!(steps >= 0.5) || steps > 1e9)
        return fail(TSK_EINVAL, "t_transient must span between one and 1e9 time steps");
    c->resolvent = true;
    c->omega = omega;
    c->ttrans = t_transient;
    c->ntrans = int(std::lround(steps));
    return TSK_OK;
}

// ---- batches: one workgroup per instance, all instances in one launch ---------------
struct CgleBatch {
    DevBuf first, second;  // job tables: V -> out (or tmp), and (M^H M) tmp -> w
    int count = 0, threads = 0, levels = 0;
    bool two = false;
};

void cgle_batch_free(CgleBatch* b) { delete b; }

tsk_status cgle_batch_plan(Operator* const* ops, int count, const KryDesc* D_host, bool svd, CgleBatchPtr* out) {
    out->reset();
    std::vector<CnJob> a(count), b(count);
    const auto* c0 = dynamic_cast<const CgleOp*>(ops[0]);
    if (!c0) return fail(TSK_EINVAL, "not a Ginzburg-Landau batch");
    for (int i = 0; i < count; ++i) {
        const auto* c = dynamic_cast<const CgleOp*>(ops[i]);
        if (!c || !c->ready()) return fail(TSK_ESTATE, "batch member is not a ready Ginzburg-Landau operator");
        if (c->nn != c0->nn) return TSK_OK;  // mixed sizes: per-instance launches
        const KryDesc& d = D_host[i];
        void* mid = svd ? ops[i]->aw.tmp.ptr : d.w;
        if (!d.V || !mid || !d.w) return fail(TSK_EINVAL, "batch workspace not allocated");
        a[i] = c->job(c->fwd, c->resolvent, c->omega);
        a[i].in = static_cast<const double2*>(d.V);
        a[i].in_stride = d.ldv;
        a[i].out = static_cast<double2*>(mid);
        if (svd) {
            b[i] = c->job(c->adj, c->resolvent, -c->omega);
            b[i].in = static_cast<const double2*>(mid);
            b[i].in_stride = 0;
            b[i].out = static_cast<double2*>(d.w);
        }
    }
    auto p = CgleBatchPtr(new CgleBatch);
    p->count = count;
    p->threads = c0->threads();
    p->levels = c0->levels;
    p->two = svd;
    TSK_TRY(p->first.ensure(sizeof(CnJob) * count));
    TSK_HIP(hipMemcpy(p->first.ptr, a.data(), sizeof(CnJob) * count, hipMemcpyHostToDevice));
    if (svd) {
        TSK_TRY(p->second.ensure(sizeof(CnJob) * count));
        TSK_HIP(hipMemcpy(p->second.ptr, b.data(), sizeof(CnJob) * count, hipMemcpyHostToDevice));
    }
    *out = std::move(p);
    return TSK_OK;
}

tsk_status cgle_batch_matvec(CgleBatch* b, int j, hipStream_t s) {
    const CnJob none{};
    TSK_TRY(launch_cn_levels(b->levels, none, b->first.as<CnJob>(), b->count, j, b->threads, s));
    if (b->two) TSK_TRY(launch_cn_levels(b->levels, none, b->second.as<CnJob>(), b->count, 0, b->threads, s));
    return TSK_OK;
}

}  // namespace tsk
