/*
 * tsk.h -- C ABI of libtsk: time-stepper Arnoldi for linear stability analysis on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Loiseau, Bucci, Cherubini & Robinet, "Time-stepping and Krylov methods
 * for large-scale instability problems", arXiv:1804.03859.
 *   - The stability of a fixed point is read from the eigenvalues of the
 *     exponential propagator M = exp(A T) (Sec. 2.2; Sec. 3.2, eq. "discrete-time
 *     linear system"); lambda = log(mu) / T.
 *   - M is never formed: one matvec M x is one time integration of the
 *     linearized equations over T (Sec. 3, "time-stepper" approach).
 *   - Ritz pairs come from the m-step Arnoldi factorisation (Sec. 3.2.1,
 *     eq. "m-step Arnoldi", Algorithm 1) and are accepted by the residual
 *     |beta e_m^T y| (Sec. 3.2.2, eq. "Krylov convergence").
 *
 * Conventions for every entry point
 *   - No exception crosses this boundary.  A negative status means nothing was
 *     written to caller buffers; tsk_last_error() then describes the failure
 *     (thread-local string, valid until the next call on the same thread).
 *   - "dev" pointers are HIP device pointers owned by the caller; "host" pointers
 *     are ordinary host memory owned by the caller.  The library never frees a
 *     caller pointer.  The operator handle and its workspace (Krylov basis,
 *     Hessenberg matrix, tables) are owned by the library until tsk_destroy().
 *   - Every operator is bound to the hipStream_t given at creation (NULL = the
 *     default stream).  tsk_apply, tsk_from_physical and tsk_to_physical are
 *     asynchronous on that stream.  tsk_arnoldi synchronises it before it writes
 *     host outputs.  The Arnoldi drivers also use three worker streams of the
 *     library's own (one set per device, shared by all operators, created on
 *     first use): Ritz analyses and the extra grid-size groups of a batched
 *     matvec run there, and every run waits for them before it returns.
 *   - A handle must not be used by two host threads at once.
 */
#ifndef TSK_H
#define TSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsk_op_s* tsk_op;

typedef enum {
    TSK_OK = 0,              /* k wanted Ritz pairs converged                      */
    TSK_NOT_CONVERGED = 1,   /* m matvecs done; outputs hold the current estimates */
    TSK_BREAKDOWN = 2,       /* invariant subspace found (beta ~ 0): pairs exact   */
    TSK_EINVAL = -1,         /* invalid argument or unsupported size               */
    TSK_ENOMEM = -2,         /* device allocation failed                           */
    TSK_EHIP = -3,           /* HIP runtime error                                  */
    TSK_ENONFINITE = -4,     /* NaN/Inf met (start vector, matvec output, beta)    */
    TSK_ESTATE = -5,         /* call out of order (e.g. parameters not set)        */
    TSK_EEIG = -6            /* Hessenberg QR did not converge                     */
} tsk_status;

typedef enum {
    TSK_FP64 = 0,            /* state, transforms and time stepping in FP64        */
    TSK_FP32 = 1             /* state in FP32; Gram-Schmidt sums, norms, H in FP64 */
} tsk_precision;

typedef struct {
    int n_matvec;            /* matvecs performed (= Arnoldi steps, Table 1 counts this way) */
    int n_ritz;              /* Ritz pairs written (k, fewer only at an early breakdown)      */
    int n_converged;         /* of those, residual <= tol                                    */
    int status;              /* same value as returned                                       */
    double beta;             /* last ||f_j||                                                 */
    double ms_total;         /* wall time of the call, host clock                            */
    double ms_apply;         /* device time of the matvecs: HIP events on the op's stream    */
                             /* around every 32nd matvec (the first included), their mean     */
                             /* times n_matvec (an event record costs stream time of its own) */
} tsk_arnoldi_info;

/* ---------------------------------------------------------------------------
 * Linear complex Ginzburg-Landau operator (Sec. 2.3.2, eq. "ginzburg-landau
 * equation"): du/dt = -nu u_x + gamma u_xx + mu(x) u, mu(x) = mu0 - c_u^2 +
 * mu2 x^2 / 2, read with nu = U + 2 i c_u and gamma = 1 + i c_d.
 * Discretised on n interior nodes of [-half_width, half_width] (dx =
 * 2 half_width/(n+1), Dirichlet ends) by second-order central differences;
 * time integration by Crank-Nicolson.  State: n complex128 values (interleaved
 * re, im), node-major.  2 <= n <= 1024.
 * ------------------------------------------------------------------------- */
tsk_status tsk_create_cgle1d(tsk_op* op, int n, double half_width, void* hip_stream);

/* dt > 0, T/dt an integer within 1e-9 relative. */
tsk_status tsk_set_params_cgle(tsk_op op, double U, double c_u, double c_d,
                               double mu0, double mu2, double dt, double T);

/* ---------------------------------------------------------------------------
 * Linearized 2D Navier-Stokes about a base flow (Sec. 3, eq. "linearized
 * Navier-Stokes equations"), vorticity form, doubly periodic box
 * [0, 2 pi/alpha) x [0, 2 pi), N x N pseudo-spectral grid with the 2/3 rule
 * (|jx|, |jy| < N/3 kept, mean mode removed), Lawson integrating-factor RK4.
 * N in {16, 32, 48, 64, 96, 128, 192, 256, 384, 512}.
 *
 * State vector ("packed spectral"): the independent real unknowns of the
 * dealiased zero-mean vorticity field, n = 4 M (M + 1) reals, M = (N-1)/3:
 *   [ kx = 0 : jy = 1..M ]  then  [ kx = j : jy = -M..M ] for j = 1..M,
 * each entry (re, im) of sqrt(2) * rfft2(omega)[jy, kx] / N^2.  With this
 * scaling the Euclidean norm of the state equals the RMS of the physical
 * field, so residuals are independent of N.  Element type: double (TSK_FP64)
 * or float (TSK_FP32).
 * Physical fields: N x N, row-major [y][x], same element type as the state.
 * ------------------------------------------------------------------------- */
tsk_status tsk_create_kolmo2d(tsk_op* op, int N, tsk_precision precision, void* hip_stream);

/* Re > 0, alpha > 0, dt > 0, T/dt an integer within 1e-9 relative. */
tsk_status tsk_set_params_kolmo(tsk_op op, double Re, double alpha, double dt, double T);

/* Parallel base flow U = (U(y), 0): host arrays of N samples at y_l = 2 pi l/N
 * of U and of dOmega/dy = -U''(y).  Copied; the caller keeps ownership. */
tsk_status tsk_set_base_parallel(tsk_op op, const double* U_y, const double* dOmega_dy);

/* Kolmogorov base flow U = (sin(n y), 0), i.e. dOmega/dy = n^2 sin(n y). */
tsk_status tsk_set_base_kolmogorov(tsk_op op, int n_forcing);

/* General 2D base flow: host arrays of N*N samples ([y][x]) of U, V and of the
 * base-vorticity gradient dOmega/dx, dOmega/dy.  Switches the operator to the
 * full two-dimensional transform pipeline. */
tsk_status tsk_set_base_flow(tsk_op op, const double* U, const double* V,
                             const double* dOmega_dx, const double* dOmega_dy);

/* Choice of the parallel-base time stepper.  0 (the default) lets the library
 * choose: for a base profile of one harmonic, U = amp sin(n (y - y0)) with
 * dOmega/dy = c U (the Kolmogorov flow sin 4y), the spectral-coupling stepper:
 * the product with one harmonic couples ky only to ky +- n, so each kx column
 * splits into n chains advanced by one wavefront each with a three-point
 * coupling and no transforms; with the 2/3 rule nothing of the pseudo-spectral
 * product wraps onto a kept mode (n < N - 2M), so it is the same operator to
 * rounding.  Otherwise the column stepper, whose kx columns per 64-lane
 * wavefront (1 or 2, 2 only for N <= 256) the library times on the first matvec
 * of a given size, precision, base kind and launch size and keeps for the
 * process.  1 or 2 force that column variant (both compute every column with
 * the same arithmetic, so results do not depend on the choice); 3 forces the
 * Bloch-sector stepper where it applies (N = 128, 256 or 512 and a profile of
 * period 2 pi / 4 with a single harmonic: each column split into the four
 * sectors ky = 4m + r, exact N/4-point products), else the column stepper.
 * tsk_get_tuning reports -2 for the spectral-coupling stepper, -1 for the
 * Bloch-sector stepper, else the forced or tuned columns per wavefront (0 = not
 * tuned yet).  Navier-Stokes operators only; TSK_EINVAL for values outside 0..3. */
tsk_status tsk_set_tuning(tsk_op op, int columns_per_wave);
tsk_status tsk_get_tuning(tsk_op op, int* columns_per_wave);

/* Launch shape of the spectral-coupling stepper: 64-lane wavefronts per
 * workgroup (1, 2 or 4; one chain per wavefront in every shape, so the results
 * are the same bits).  0 (the default) lets the library time the three shapes
 * on the first launch of a given precision, chain layout and launch size (a
 * single matvec, or a batch's shared launch) and keep the fastest for the
 * process.  tsk_get_stepper_waves reports the forced shape, else the shape of
 * the operator's last single matvec (0 before the first).  Navier-Stokes
 * operators only; TSK_EINVAL for other values. */
tsk_status tsk_set_stepper_waves(tsk_op op, int waves_per_group);
tsk_status tsk_get_stepper_waves(tsk_op op, int* waves_per_group);

/* Stop rule of the Arnoldi stop test (Sec. 3.2.2, eq. "Krylov convergence":
 * a Ritz pair is converged when |beta e_m^T y| <= tol), per operator, for
 * tsk_arnoldi, tsk_batch_arnoldi and tsk_krylov_schur:
 *   res_floor_rel: a pair also counts as converged once its estimate is below
 *                  res_floor_rel |mu| (converged: res <= max(tol, res_floor_rel |mu|)).
 *   dup_rel:       Ritz values closer than dup_rel |mu| to an accepted value are
 *                  copies of one eigenvalue (the duplicate width of the wanted set).
 * A negative value restores the default of the state type: FP64 states 0 and 0
 * (the plain rule); FP32 states 32 u32 = 1.9e-6 and 2e-5, because the FP32
 * basis holds the Arnoldi relation only to about u32 ||M|| and FP32 rounding
 * splits multiple eigenvalues into clusters.  res_floor_rel = 0 makes an FP32
 * run stop on the same estimate <= tol as an FP64 run.  Values must be finite
 * and below 1e-2 (TSK_EINVAL otherwise). */
tsk_status tsk_set_stop_rule(tsk_op op, double res_floor_rel, double dup_rel);

/* ---------------------------------------------------------------------------
 * Common to all operators.
 * ------------------------------------------------------------------------- */

/* n_scalars: state length in scalars (complex count if *is_complex);
 * elem_bytes: bytes per real component (8 or 4). */
tsk_status tsk_state_dim(tsk_op op, int64_t* n_scalars, int* is_complex, int* elem_bytes);

/* Physical field (dev) -> state (dev): orthogonal projection on the state
 * space (for the Navier-Stokes operator: dealias and drop the mean).  For the
 * Ginzburg-Landau operator the two representations coincide (a copy). */
tsk_status tsk_from_physical(tsk_op op, const void* phys_dev, void* state_dev);

/* State (dev) -> physical field (dev). */
tsk_status tsk_to_physical(tsk_op op, const void* state_dev, void* phys_dev);

/* One matvec y = M x = (time integration over T) x.  x and y are state vectors
 * in device memory; they may not alias. */
tsk_status tsk_apply(tsk_op op, const void* x_dev, void* y_dev);

/* y = M^dagger x: the adjoint propagator, the transpose (conjugate transpose for
 * complex states) of the discrete propagator of tsk_apply in the state's
 * Euclidean inner product (Sec. 2.2: for the Euclidean inner product the
 * adjoint is the conjugate transpose; Sec. 3.3.2: M^dagger is one backward
 * integration of the adjoint system).  Navier-Stokes operators: each IF-RK4
 * step transposed stage by stage, for parallel base flows (the transposed
 * steppers) and for a general 2-D base flow after tsk_set_base_flow (the
 * transposed two-dimensional pipeline: one inverse and four forward transforms
 * per stage).  Ginzburg-Landau: Crank-Nicolson on L_h^H.  Same layout, stream
 * and aliasing rule as tsk_apply. */
tsk_status tsk_apply_adjoint(tsk_op op, const void* x_dev, void* y_dev);

/* Resolvent mode (Sec. 2.3.2; Sec. 3.3.2, the resolvent by forced time
 * integration) of a Ginzburg-Landau operator: tsk_apply(op, f, x) then returns
 * x^ = R(omega) f^, the asymptotic response to the forcing f^ e^{i omega t}:
 * Crank-Nicolson from rest over t_transient time units (forcing by the
 * trapezoidal rule), read as u(t) e^{-i omega t} (the response is a single
 * harmonic, so this is its Fourier coefficient).  It is the resolvent of the
 * discrete L_h at the warped frequency (2/dt) tan(omega dt/2), up to the
 * transient remainder (decay rate: the least stable eigenvalue; the system must
 * be stable).  tsk_apply_adjoint returns R(omega)^H (L_h^H at -omega), so
 * tsk_optimal_perturbation gives the resolvent gains sigma^2 and the optimal
 * forcings.  t_transient = 0 returns to the propagator.  TSK_EINVAL for other
 * operators (the complex forcing needs a complex state). */
tsk_status tsk_set_resolvent(tsk_op op, double omega, double t_transient);

/* Optimal perturbation (Sec. 2.3.1, SVD formulation; Sec. 3.3.2): the k largest
 * singular values sigma of M = exp(A T) by the Lanczos iteration on the
 * symmetric M^dagger M.  Each step is one forward and one adjoint integration,
 * classical Gram-Schmidt twice against every previous vector (full
 * reorthogonalisation), and a device symmetric tridiagonal QR for the Ritz
 * values theta = sigma^2.  Wanted set, residual (|beta e_m^T y| of the
 * M^dagger M eigenpair), tolerance and stop rule as tsk_arnoldi.  The optimal
 * gain over T is sigma_1^2.
 *   m, k, tol, v0_dev, seed: as tsk_arnoldi (1 <= k <= m <= 96).
 *   sigma:    host, k doubles, descending (the wanted order).
 *   resid:    host, k doubles.
 *   vecs_dev: dev or NULL: the k right singular vectors (optimal initial
 *             conditions), unit norm, each n complex128 (imaginary part zero
 *             for real operators), vector-major; the responses are M x = sigma u.
 *   info:     host or NULL; n_matvec counts Lanczos steps (two integrations each).
 * Returns TSK_OK, TSK_NOT_CONVERGED or TSK_BREAKDOWN with outputs written, or a
 * negative status with nothing written (TSK_EINVAL when the operator has no
 * adjoint). */
tsk_status tsk_optimal_perturbation(tsk_op op, int m, int k, double tol, const void* v0_dev, uint64_t seed,
                                    double* sigma, double* resid, void* vecs_dev, tsk_arnoldi_info* info);

/* Batched optimal perturbation / resolvent gains (Sec. 2.3.1, 2.3.2; Sec.
 * 3.3.2), for sweeps over target times or forcing frequencies: `count`
 * operators of one state type and one stream, each with an adjoint, advance
 * their Lanczos iterations in lockstep; the integrations of Ginzburg-Landau
 * instances of one node count (the resolvent of each at its own frequency, or
 * its propagator) run in one launch per pass, one workgroup per instance.  Each
 * instance stops on its own test.  Arguments as for tsk_optimal_perturbation,
 * per instance i: v0_devs[i] (array or entries may be NULL), seeds[i] (NULL
 * array: seed i), sigma + k i, resid + k i, vecs_devs[i] (array or entries may
 * be NULL), infos[i] (per-instance status).  Returns TSK_OK when every instance
 * ended without error (see infos[i].status), or a negative status for an
 * argument or runtime failure of the whole batch. */
tsk_status tsk_batch_optimal_perturbation(const tsk_op* ops, int count, int m, int k, double tol,
                                          const void* const* v0_devs, const uint64_t* seeds, double* sigma,
                                          double* resid, void* const* vecs_devs, tsk_arnoldi_info* infos);

/* Arnoldi with classical Gram-Schmidt applied twice (Sec. 3.2.1, Algorithm 1),
 * Ritz pairs from a device-side Hessenberg QR after every matvec, stop when the
 * k wanted pairs have |beta e_m^T y| <= tol (Sec. 3.2.2), or after m matvecs,
 * or at a happy breakdown.
 *   m:        maximum Krylov dimension, 1 <= k <= m <= 96, m <= state length.
 *   tol:      residual tolerance (absolute, unit-norm Ritz vectors); 0 = run m.
 *   v0_dev:   start vector (state, dev) or NULL: then an iid N(0,1) field drawn
 *             from `seed` (splitmix64 + Box-Muller, counter = element index of
 *             the physical field) is projected on the state space.
 *   mu_ri:    host, 2k doubles: Ritz values of M (re, im), wanted order.
 *   lambda_ri:host, 2k doubles: log(mu)/T, principal branch.
 *   resid:    host, k doubles: residual estimates.
 *   ritz_dev: dev or NULL: k Ritz vectors V y, each n complex128 (interleaved),
 *             vector-major.
 *   info:     host or NULL.
 * Returns TSK_OK, TSK_NOT_CONVERGED or TSK_BREAKDOWN with outputs written, or a
 * negative status with nothing written. */
tsk_status tsk_arnoldi(tsk_op op, int m, int k, double tol, const void* v0_dev, uint64_t seed,
                       double* mu_ri, double* lambda_ri, double* resid, void* ritz_dev,
                       tsk_arnoldi_info* info);

/* Batched Arnoldi (neutral-curve sweeps): `count` operators of one state type
 * and one stream (for example Navier-Stokes operators of different N, Re and
 * alpha, all FP32) advance in lockstep; the matvecs of all Navier-Stokes
 * instances of one grid size run in one launch.  Each instance stops on its
 * own test; the call returns when all have stopped.  Arguments as for
 * tsk_arnoldi, per instance i: v0_devs[i] (array or entries may be NULL),
 * seeds[i] (NULL array: seed i), mu_ri + 2k i, lambda_ri + 2k i, resid + k i,
 * ritz_devs[i] (array or entries may be NULL), infos[i] (per-instance status).
 * Returns TSK_OK when every instance ended without error (see infos[i].status),
 * or a negative status for an argument or runtime failure of the whole batch. */
tsk_status tsk_batch_arnoldi(const tsk_op* ops, int count, int m, int k, double tol,
                             const void* const* v0_devs, const uint64_t* seeds, double* mu_ri,
                             double* lambda_ri, double* resid, void* const* ritz_devs,
                             tsk_arnoldi_info* infos);

/* Krylov-Schur run statistics. */
typedef struct {
    int n_matvec;            /* matvecs: m, plus m - p per contraction (Table 1 counts this way) */
    int n_restarts;          /* contractions performed                                          */
    int n_ritz;              /* Ritz pairs written (k, fewer only at an early breakdown)         */
    int n_converged;         /* of those, residual <= tol                                        */
    int status;              /* same value as returned                                           */
    int kept_last;           /* order p kept by the last contraction (0: none)                  */
    double beta;             /* residual norm of the final factorisation                          */
    double ms_total;         /* wall time of the call, host clock                                 */
    double ms_apply;         /* device time of the matvecs, HIP events on the op's stream         */
} tsk_ks_info;

/* Krylov-Schur method (Sec. 3.2.2, after Stewart 2001) for real operators.
 * Expand an Arnoldi factorisation (classical Gram-Schmidt twice) to order m;
 * test the k wanted Ritz pairs with the wanted set, residual and tolerance of
 * tsk_arnoldi, at order m only (steps 2 and 6 of the method); while the test
 * fails, order the real Schur form of H_m so that the kept Ritz values lead,
 * truncate to their order p and expand again from v_{p+1} = v_{m+1}.  The
 * truncated Krylov-Schur decomposition is brought back to an equivalent
 * Arnoldi factorisation (same Ritz pairs) before the expansion continues.
 *   m:            Krylov dimension, k + 2 <= m <= 96, m <= state length.
 *   k, tol:       as tsk_arnoldi.
 *   delta:        a contraction keeps the Ritz values with |mu| >= 1 - delta
 *                 (the paper uses 0.05 to 0.1) ...
 *   p_max:        ... but at least k and at most p_max of them, the leading
 *                 ones by |mu| (k <= p_max <= m - 2; 0 selects max(k, m / 2));
 *                 a complex pair is kept whole, so p may be p_max + 1.
 *   max_restarts: contractions allowed before returning TSK_NOT_CONVERGED.
 *   v0_dev, seed, mu_ri, lambda_ri, resid, ritz_dev, as tsk_arnoldi.
 * Returns TSK_OK, TSK_NOT_CONVERGED or TSK_BREAKDOWN with outputs written, or a
 * negative status with nothing written (TSK_EINVAL also for complex operators,
 * TSK_EEIG if the QR iteration or the reordering failed). */
tsk_status tsk_krylov_schur(tsk_op op, int m, int k, double tol, double delta, int p_max, int max_restarts,
                            const void* v0_dev, uint64_t seed, double* mu_ri, double* lambda_ri, double* resid,
                            void* ritz_dev, tsk_ks_info* info);

/* Batched Krylov-Schur for neutral-curve sweeps (Sec. 3.2.2): `count` real
 * operators (one state type and one stream) advance in lockstep as in
 * tsk_batch_arnoldi, with the Ritz analysis and stop test after every matvec,
 * up to order m.  Every instance still not converged at order m then continues
 * as tsk_krylov_schur does: contraction to its kept Ritz values (|mu| >= 1 -
 * delta, raised to k and lowered to p_max), rotation of its basis, expansion
 * back to order m, test at order m, at most max_restarts contractions.  The
 * contractions of all such instances run in one launch (one wavefront each) and
 * their expansions in lockstep, instance i from its own kept order.  Arguments
 * as tsk_batch_arnoldi (per instance i: v0_devs[i], seeds[i], mu_ri + 2k i,
 * lambda_ri + 2k i, resid + k i, ritz_devs[i]) and tsk_krylov_schur (delta,
 * p_max: 0 = max(k, m/2), max_restarts); infos[i] (host array or NULL): the
 * instance's matvecs (m + (m - p) per contraction when it restarted), its
 * contractions and status; ms_apply times the matvecs of the lockstep phase
 * (the expansion of a restart cycle of one shared matvec launch per step runs as
 * one captured HIP graph and is not timed per matvec).  Returns TSK_OK when every instance ended without
 * error (see infos[i].status), or a negative status for an argument or runtime
 * failure of the whole batch. */
tsk_status tsk_batch_krylov_schur(const tsk_op* ops, int count, int m, int k, double tol, double delta, int p_max,
                                  int max_restarts, const void* const* v0_devs, const uint64_t* seeds, double* mu_ri,
                                  double* lambda_ri, double* resid, void* const* ritz_devs, tsk_ks_info* infos);

/* The contraction on its own (the device kernel tsk_krylov_schur runs at
 * order m).  Input: H_dev, m x m real upper Hessenberg (FP64, column-major,
 * leading dimension ldh >= m; only the Hessenberg part is read), and beta, the
 * residual norm of its Arnoldi factorisation.  Kept set from k, delta and p_max
 * as tsk_krylov_schur (k + 2 <= m <= 96).  Outputs (device):
 *   mu_dev:   m complex128, the Ritz values of H (real Schur order);
 *   res_dev:  m doubles, their residuals beta |e_m^T y|, unit y;
 *   Hnew_dev: (m+1) x m FP64, column-major, leading dimension m+1: the new
 *             Hessenberg H_p in rows 0..p-1 of columns 0..p-1, beta' >= 0 at
 *             (p, p-1), zero elsewhere;
 *   W_dev:    room for m x m FP64; its first p columns (leading dimension m)
 *             receive the orthonormal W with V_p = V_m W.
 * Host outputs: *kept = p, *beta_new = beta'.  Synchronous on hip_stream.
 * TSK_EEIG if the QR iteration or the reordering failed, TSK_ENONFINITE if H
 * or beta is not finite. */
tsk_status tsk_ks_contract(const double* H_dev, int ldh, int m, double beta, int k, double delta, int p_max,
                           void* mu_dev, double* res_dev, double* Hnew_dev, double* W_dev, int* kept,
                           double* beta_new, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Fixed points (Sec. 3.1).  A Navier-Stokes operator also carries the
 * nonlinear forced equation
 *     d omega/dt + (u + U0) d_x omega + v d_y omega = Re^-1 lap omega + f
 * on the same grid, state space and time scheme as its linearized matvec
 * (u = d_y psi, v = -d_x psi, -lap psi = omega; U0 a uniform drift along x).
 * f = -Re^-1 lap omega_lam holds the laminar Kolmogorov flow omega_lam =
 * -n cos(n y) steady; an optional extra forcing field makes the steady state
 * two-dimensional.  The discrete-time system is x_{k+1} = G(x_k), G = T/dt
 * steps.  On success every solver below leaves the operator's base flow set to
 * the fixed point found (tsk_set_base_from_state), so tsk_arnoldi then gives
 * its stability (the paper's fixed point -> eigenvalues workflow).
 * ------------------------------------------------------------------------- */
typedef struct {
    int status;              /* same value as returned                                     */
    int iterations;          /* outer iterations (SFD: residual checks)                     */
    int64_t time_steps;      /* nonlinear time steps taken                                  */
    int basis_dim;           /* RPM: unstable basis size p; BoostConv: pairs in the history */
    double residual;         /* last residual: ||G(x) - x|| (SFD: ||step(x) - x|| / dt)     */
    double ms_total;         /* wall time of the call, host clock                           */
} tsk_fp_info;

/* Set up the nonlinear equation (after tsk_set_params_kolmo; re-derived when
 * the parameters change).  n_forcing in [1, (N-1)/3]; extra_forcing: host N*N
 * physical field ([y][x], FP64) projected on the state space, or NULL. */
tsk_status tsk_set_nonlinear(tsk_op op, int n_forcing, double U0, const double* extra_forcing);
/* The packed laminar state omega_lam (dev). */
tsk_status tsk_laminar_state(tsk_op op, void* x_dev);
/* y = nsteps Lawson IF-RK4 steps of the nonlinear equation from x (dev states;
 * nsteps = 0: T/dt steps, i.e. G(x)).  x and y may not alias. */
tsk_status tsk_nonlinear_step(tsk_op op, const void* x_dev, void* y_dev, int nsteps);
/* The operator's (general two-dimensional) base flow becomes the state x: its
 * grid fields (u + U0, v, grad omega) computed on the device.  tsk_apply then
 * is the Jacobian of the nonlinear stepper's right-hand side about x. */
tsk_status tsk_set_base_from_state(tsk_op op, const void* x_dev);
/* Selective frequency damping (Sec. 3.1.1; Akervik et al. 2006): the extended
 * system X' = F(X) - chi (X - Y), Y' = (X - Y)/Delta, Strang-split per time step
 * (exact coupling over dt/2, one nonlinear step, coupling over dt/2).  x_dev:
 * start (in), result (out).  Every check_every steps the residual
 * ||step(X) - X|| / dt is taken (history in hist[max_checks] if not NULL); stop
 * when <= tol.  It cannot quench non-oscillating instabilities. */
tsk_status tsk_sfd(tsk_op op, void* x_dev, double chi, double delta, int check_every, double tol, int max_checks,
                   double* hist, tsk_fp_info* info);
/* Recursive projection method (Sec. 3.1.2; Shroff & Keller 1993): U, H = U^T M U
 * from an m-step Arnoldi factorisation of the Jacobian about the start (started
 * from the initial residual) contracted to its Ritz values |mu| >= 1 - delta (at
 * least k) by the Krylov-Schur kernel; then x~ <- G(x~) - U U^T r + U (I - H)^-1 U^T r,
 * r = G(x~) - x~, until ||r|| <= tol (history in hist[max_iter]).  1 <= k,
 * k + 2 <= m <= 96. */
tsk_status tsk_rpm(tsk_op op, void* x_dev, int m, int k, double delta, double tol, int max_iter, double* hist,
                   tsk_fp_info* info);
/* BoostConv (Sec. 3.1.3; Citro et al. 2017): with the corrections xi_j and the
 * residual decrements r_j - r_{j+1} of the last m iterations (1 <= m <= 96),
 * c = (Y^T Y)^-1 Y^T r, x~ <- x~ + r + (X - Y) c, until ||r|| <= tol. */
tsk_status tsk_boostconv(tsk_op op, void* x_dev, int m, double tol, int max_iter, double* hist, tsk_fp_info* info);

/* Last Arnoldi run, for inspection: H ((m+1) x m complex128, column-major,
 * leading dimension m+1, zero beyond the steps taken) copied to host, and the
 * basis pointer (device, (steps+1) vectors of the state type, vector-major,
 * stride *ld elements).  Valid until the next tsk_arnoldi or tsk_destroy. */
tsk_status tsk_last_hessenberg(tsk_op op, double* H_host, int* m_out, int* steps_out);
tsk_status tsk_last_basis(tsk_op op, const void** V_dev, int64_t* ld);

/* Device Hessenberg eigensolver on its own (the one tsk_arnoldi uses):
 * H_dev: p x p complex128 upper Hessenberg, column-major with leading
 * dimension ldh (>= p); beta: residual scale.  Outputs (dev): mu_dev (p
 * complex128), Y_dev (p x p complex128, column-major, unit-norm columns),
 * res_dev (p doubles, beta |Y[p-1, i]|).  1 <= p <= 96.  Synchronous on
 * hip_stream.  Returns TSK_EEIG if the QR iteration failed to converge and
 * TSK_ENONFINITE (outputs not written) if H or beta holds a NaN or Inf. */
tsk_status tsk_hessenberg_ritz(const void* H_dev, int ldh, int p, double beta,
                               void* mu_dev, void* Y_dev, void* res_dev, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Learned start vector (not part of the paper).  Algorithm 1 (Sec. 3.2.1)
 * takes any start vector; one close to the wanted invariant subspace shortens
 * the Krylov sequence.  A three-layer perceptron maps (Re, alpha) of a
 * Navier-Stokes operator with a parallel base flow to the 32 x 32 block of low
 * Fourier coefficients jx in [0, 32), jy in [-16, 16) of the packed state: 2048
 * reals, index 2 (32 jx + jy + 16) + c (c = 0 re, 1 im).  Block positions that
 * a state does not hold (jx = 0 with jy <= 0; |jx| or |jy| > M) are ignored.
 *
 * Network: x = 2 (p - in_lo) / (in_hi - in_lo) - 1 for p = (Re, alpha);
 * A1 = tanh(x W1 + b1), A2 = tanh(A1 W2 + b2), Y = A2 W3 + b3, width W.
 * FP32 master parameters, flat layout W1 [2][W], b1 [W], W2 [W][W], b2 [W],
 * W3 [W][2048], b3 [2048] (weights row-major [in][out]), 2048 + W (W + 2052)
 * floats.  Layers 2 and 3 and their backward products use bfloat16 copies of
 * weights and activations (round to nearest even) with FP32 accumulation on
 * the matrix cores.  Loss L = sum (Y - target)^2 / (batch 2048).  Training is
 * full-batch Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * The network runs on its own stream (NULL = default), except tsk_mlp_start,
 * which runs on the operator's stream after waiting for the network's.
 * ------------------------------------------------------------------------- */
typedef struct tsk_mlp_s* tsk_mlp;
/* width: multiple of 16 in [16, 2048] (512 for the learned start).
 * in_lo/in_hi: host, 2 doubles each: the (Re, alpha) box mapped onto [-1, 1]^2. */
tsk_status tsk_mlp_create(tsk_mlp* net, int width, const double* in_lo, const double* in_hi, void* hip_stream);
tsk_status tsk_mlp_param_count(tsk_mlp net, int64_t* count);
/* Xavier-uniform weights (element e of the flat vector from splitmix64 output e
 * of `seed`: u = (o >> 11) 2^-53, w = l (2u - 1), l = sqrt(6/(fan_in+fan_out))),
 * zero biases; resets the optimizer. */
tsk_status tsk_mlp_init(tsk_mlp net, uint64_t seed);
/* Host copies of the flat FP32 parameters; set resets the optimizer. */
tsk_status tsk_mlp_set_params(tsk_mlp net, const float* params_host);
tsk_status tsk_mlp_get_params(tsk_mlp net, float* params_host);
/* in_dev: batch x 2 floats (Re, alpha); out_dev: batch x 2048 floats.
 * 1 <= batch <= 4096.  Asynchronous on the network's stream. */
tsk_status tsk_mlp_forward(tsk_mlp net, const float* in_dev, int batch, float* out_dev);
/* Loss and full gradient (flat layout, dev, may be NULL) without an update. */
tsk_status tsk_mlp_gradients(tsk_mlp net, const float* in_dev, const float* target_dev, int batch,
                             float* grad_dev, double* loss_host);
/* `steps` full-batch Adam steps with learning rate lr; loss_host (NULL or
 * `steps` doubles) receives the loss before each update. */
tsk_status tsk_mlp_train(tsk_mlp net, const float* in_dev, const float* target_dev, int batch, int steps,
                         double lr, double* loss_host);
/* Training target (2048 floats, dev) from k Ritz vectors of a Navier-Stokes
 * operator (ritz_dev as written by tsk_arnoldi; use_host: k flags or NULL =
 * all).  Per used vector: its real part (imaginary part if larger), block
 * coefficients, canonical x-translation making the largest coefficient real
 * positive (sign only when it sits at jx = 0; ties within 1e-6 relative go to
 * the lowest slot), unit norm; the sum is scaled to unit norm (zero if no
 * vector had block content).  Synchronous on the operator's stream. */
tsk_status tsk_ritz_block_target(tsk_op op, const void* ritz_dev, int k, const int* use_host,
                                 float* target_dev);
/* Start vector (state, dev) for a Navier-Stokes operator: the prediction p for
 * (Re, alpha) scattered into the state, v0 = p/||p|| + gamma r/||r|| with r the
 * seeded random state of tsk_arnoldi; the random start r/||r|| alone when ||p||
 * is zero or not finite (*used_net = 0, else 1).  gamma >= 0. */
tsk_status tsk_mlp_start(tsk_mlp net, tsk_op op, double Re, double alpha, double gamma, uint64_t seed,
                         void* v0_dev, int* used_net);
void tsk_mlp_destroy(tsk_mlp net);

/* The real-arithmetic solver tsk_arnoldi uses for real operators (Francis
 * double-shift QR, Golub & Van Loan Algorithms 7.5.1-7.5.2): H_dev is p x p
 * real FP64, column-major with leading dimension ldh (>= p); only its upper
 * Hessenberg part is read.  Outputs (dev): mu_dev (p complex128: eigenvalues,
 * a complex pair as (a + ib, a - ib) in consecutive entries), res_dev (p doubles:
 * beta |e_p^T y| for the unit eigenvector y of each eigenvalue).  1 <= p <= 96.
 * Synchronous on hip_stream.  TSK_EEIG if the iteration failed to converge,
 * TSK_ENONFINITE if H or beta holds a NaN or Inf. */
tsk_status tsk_hessenberg_ritz_real(const double* H_dev, int ldh, int p, double beta, void* mu_dev,
                                    void* res_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solver and outputs as tsk_hessenberg_ritz_real, with its scratch (a complex
 * copy of H, the eigenvector workspace, the result record, device scalars, the
 * solver's descriptor) in a fixed device array of 297 KB that the library keeps
 * on every GPU it runs on until the process ends, instead of allocations per
 * call.  The caller still passes H and the outputs.  Limits of that array:
 * 1 <= p <= 96 and p <= ldh <= 97 (TSK_EINVAL beyond them).  The call makes no
 * device allocation or free.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two host threads, or two streams) race, and
 * each call rewrites what it needs before the solve.  Synchronous on
 * hip_stream; same status codes as tsk_hessenberg_ritz_real. */
tsk_status tsk_hessenberg_ritz_real_noalloc(const double* H_dev, int ldh, int p, double beta, void* mu_dev,
                                            void* res_dev, void* hip_stream);
/* iid N(0,1) draws (device, FP64): count values of the splitmix64 +
 * Box-Muller stream of `seed` (element e uses outputs 2*(e/2), 2*(e/2)+1). */
tsk_status tsk_normal_fill(double* out_dev, int64_t count, uint64_t seed, void* hip_stream);

void tsk_destroy(tsk_op op);
const char* tsk_status_str(int status);
const char* tsk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSK_H */
