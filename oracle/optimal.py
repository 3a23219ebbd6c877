"""Oracle: adjoint propagators and optimal perturbations (leading singular values
of M) by the Lanczos iteration on M^dagger M.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper:
* Sec. 2.3.1, "Formulation using SVD": the optimal energy gain over a target time
  T is G(T) = max ||M x0||^2 / ||x0||^2 = sigma_1^2, sigma_1 the largest
  singular value of M = exp(A T); the optimal initial condition is the principal
  right singular vector and the response at T is sigma_1 times the principal
  left singular vector.
* Sec. 2.2 (footnote on the adjoint): for the Euclidean inner product the
  adjoint operator is the conjugate transpose.
* Sec. 3.3.2, "Singular value decomposition": M^dagger M v = sigma^2 v; the action
  of M^dagger M is a forward integration followed by an adjoint integration;
  since M^dagger M is symmetric positive definite, the Hessenberg matrix of the
  Arnoldi iteration becomes tridiagonal, i.e. the Lanczos iteration (Lanczos
  1950).

Readings (where the paper leaves a choice open):
* The adjoint is the discrete adjoint: the transpose (conjugate transpose for
  complex states) of the discrete propagator in the state's Euclidean inner
  product, so M^dagger M is symmetric to rounding.  Kolmogorov flow: each Lawson
  IF-RK4 step is transposed stage by stage (reverse order) with the transposed
  advection operator.  The transpose of -P(U d_x + V d_y + Omega_x d_y L -
  Omega_y d_x L)P on the dealiased subspace is P(d_x U + d_y V + L d_y Omega_x -
  L d_x Omega_y)P, because the spectral derivatives are skew, the grid products
  and L = lap^-1 (multiplier 1/K^2) are symmetric and P is an orthogonal
  projector.  Ginzburg-Landau: Crank-Nicolson applied to L_h^H, which is the
  conjugate transpose of the Crank-Nicolson propagator of L_h because the two
  factors of a step commute.
* Lanczos with full reorthogonalisation: every new vector is projected twice
  (classical Gram-Schmidt) against all previous ones, as in the Arnoldi oracle.
  The tridiagonal T_j takes alpha_j = the coefficient on v_j and beta_j = the
  norm of the projected vector; the other projection coefficients are
  rounding-level reorthogonalisation corrections and are dropped.
* Ritz pairs from LAPACK eigh of T_j, residual |beta_j y_j| for unit y, wanted
  set and stop test of the Arnoldi oracle (values theta = sigma^2 are real).
  One Lanczos step costs one forward and one adjoint integration.
* Norm: the state's Euclidean norm (for the vorticity state, the enstrophy).

Parity status: pinned (dot-product identity <M x, y> = <x, M^dagger y> and the
dense transpose on tiny grids; Lanczos against LAPACK svd/eigh of dense
matrices; the Schmid 2x2 system's closed-form singular values; the dense SVD of
the assembled Kolmogorov and Ginzburg-Landau propagators); see
tests/test_oracle_optimal.py.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded

from oracle.arnoldi import BREAKDOWN, NOT_CONVERGED, OK, select_wanted

EPS = np.finfo(float).eps


# ---- Kolmogorov flow: transposed advection and reversed IF-RK4 --------------------
def kolmo_advection_transpose(op, zh):
    """Transpose of op.advection_hat on the dealiased subspace (masked rfft2 in and
    out): P(d_x U + d_y V + L d_y Omega_x - L d_x Omega_y)P, products on the grid."""
    z = op.to_physical(zh * op.mask)
    rf = lambda f: np.fft.rfft2(f) * op.mask
    g1, g2 = rf(op.U * z), rf(op.V * z)
    g3, g4 = rf(op.Ox * z), rf(op.Oy * z)
    return op.mask * (1j * op.kx * g1 + 1j * op.ky * g2 + op.invK2 * (1j * op.ky * g3 - 1j * op.kx * g4))


def kolmo_step_transpose(op, zh):
    """Transpose of one Lawson IF-RK4 step (op.step_hat).  With the forward stages
    a = N w, b = N E_h (w + h/2 a), c = N (E_h w + h/2 b), d = N (E_1 w + h E_h c),
    w+ = E_1 w + h/6 (E_1 a + 2 E_h (b + c) + d), the reverse sweep from z = w+bar is
    d' = h/6 z, s3 = N^T d', c' = h/3 E_h z + h E_h s3, s2 = N^T c',
    b' = h/3 E_h z + h/2 s2, s1 = N^T b', a' = h/6 E_1 z + h/2 E_h s1, s0 = N^T a',
    w-bar = E_1 z + E_1 s3 + E_h s2 + E_h s1 + s0 (E diagonal and real)."""
    h = op.dt
    E1 = np.exp(-op.K2 * h / op.Re)
    Eh = np.exp(-op.K2 * (h / 2) / op.Re)
    Nt = lambda v: kolmo_advection_transpose(op, v)
    s3 = Nt((h / 6) * zh)
    s2 = Nt((h / 3) * Eh * zh + h * Eh * s3)
    s1 = Nt((h / 3) * Eh * zh + (h / 2) * s2)
    s0 = Nt((h / 6) * E1 * zh + (h / 2) * Eh * s1)
    return E1 * zh + E1 * s3 + Eh * s2 + Eh * s1 + s0


def kolmo_apply_adjoint(op, z):
    """M^T z for the Kolmogorov propagator: physical field in, physical field out
    (the grid inner product on the dealiased subspace)."""
    zh = op.to_spectral(z)
    for _ in range(op.nsteps):
        zh = kolmo_step_transpose(op, zh)
    return op.to_physical(zh)


# ---- Ginzburg-Landau: Crank-Nicolson on L_h^H --------------------------------------
def cgle_apply_adjoint(op, u):
    """M^H u for the Crank-Nicolson propagator of L_h: T/dt steps of
    (I - dt/2 L^H) u+ = (I + dt/2 L^H) u, L^H = conj(L) transposed."""
    sub, main, sup = op.bands()
    sub_h, main_h, sup_h = np.conj(sup), np.conj(main), np.conj(sub)
    h = 0.5 * op.dt
    ab = np.zeros((3, op.n), dtype=complex)
    ab[0, 1:] = -h * sup_h
    ab[1, :] = 1.0 - h * main_h
    ab[2, :-1] = -h * sub_h
    u = np.asarray(u, dtype=complex).copy()
    for _ in range(op.nsteps):
        r = main_h * u
        r[1:] += sub_h * u[:-1]
        r[:-1] += sup_h * u[1:]
        u = solve_banded((1, 1), ab, u + h * r)
    return u


# ---- Lanczos iteration -------------------------------------------------------------
def lanczos(apply_A, v0, m, k, tol, keep_basis=True):
    """Lanczos with full reorthogonalisation on a symmetric (Hermitian) operator.

    Returns theta, res (k wanted), X (Ritz vectors n x k), sel, n_steps, status,
    alpha, beta and the basis V."""
    v0 = np.asarray(v0).ravel()
    n = v0.size
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= m")
    nrm0 = np.sqrt(np.vdot(v0, v0).real)
    if not np.isfinite(nrm0) or nrm0 == 0.0:
        raise ValueError("start vector must be finite and non-zero")
    dtype = np.result_type(v0.dtype, np.float64)
    V = np.zeros((m + 1, n), dtype=dtype)
    V[0] = v0 / nrm0
    alpha = np.zeros(m)
    beta = np.zeros(m)
    status = NOT_CONVERGED
    theta = Y = res = None
    sel = []
    j_done = 0
    for j in range(m):
        w = np.asarray(apply_A(V[j].copy()), dtype=dtype).ravel()
        w_in = np.sqrt(np.vdot(w, w).real)
        Vj = V[: j + 1]
        h1 = Vj.conj() @ w
        w = w - Vj.T @ h1
        h2 = Vj.conj() @ w
        w = w - Vj.T @ h2
        alpha[j] = (h1 + h2)[j].real
        beta[j] = np.sqrt(np.vdot(w, w).real)
        j_done = j + 1
        T = np.diag(alpha[: j + 1]) + np.diag(beta[:j], 1) + np.diag(beta[:j], -1)
        theta, Y = np.linalg.eigh(T)
        res = np.abs(beta[j] * Y[-1, :])
        kk = min(k, j + 1)
        sel, done = select_wanted(theta.astype(complex), res, kk, tol, 1.0)
        if beta[j] <= 64 * EPS * w_in:
            status = BREAKDOWN
            break
        if done and kk == k:
            status = OK
            break
        V[j + 1] = w / beta[j]
    p = j_done
    X = V[:p].T @ Y[:, sel]
    out = dict(theta=theta[sel], res=res[sel], X=X, sel=sel, n_steps=p, status=status,
               alpha=alpha[:p].copy(), beta=beta[:p].copy(), all_theta=theta, all_res=res)
    if keep_basis:
        out["V"] = V[: p + 1]
    return out


def optimal_perturbation(apply, apply_adjoint, v0, m, k, tol):
    """Leading singular values of M (Sec. 3.3.2): Lanczos on M^dagger M.
    Returns a dict with sigma (k), gain = sigma^2, res (residuals of the
    M^dagger M eigenpairs), X (right singular vectors, n x k, unit norm) and the
    Lanczos statistics."""
    r = lanczos(lambda v: apply_adjoint(apply(v)), v0, m, k, tol)
    r["gain"] = r["theta"]
    r["sigma"] = np.sqrt(np.maximum(r["theta"], 0.0))
    return r
