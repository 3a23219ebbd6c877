"""Oracle: m-step Arnoldi factorisation on a black-box matvec, Ritz pairs, residual
estimates, wanted set / stop rule and the continuous-time eigenvalues.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper:
* Sec. 3.2 eq. "discrete-time linear system": x_{k+1} = M x_k with
  M = exp(A T); the system is unstable iff some |mu| > 1; lambda = log(mu)/T.
* Sec. 3.2.1, eq. "m-step Arnoldi" and Algorithm 1: M V_m = V_m H_m + r_m e_m^T,
  v1 = v/||v||, w = M v_j, h = V^T w, f = w - V h, beta = ||f||,
  v_{j+1} = f/beta, H grows by one column per matvec.  Ritz pairs
  (mu_H, V_m y) approximate eigenpairs of M.  The Nyquist remark (at least four
  samples per period) is why the principal branch of log is used.
* Sec. 3.2.2, eq. "Krylov convergence": ||M V y - mu V y|| = |beta e_m^T y|;
  a Ritz pair counts as converged when that residual is below a tolerance.

Readings (where the paper is silent or inconsistent):
* Orthogonalisation: Algorithm 1 projects once with classical Gram-Schmidt (the
  comparison section calls it modified Gram-Schmidt); here classical Gram-Schmidt
  is applied twice (CGS2) and H's new column is h1 + h2.
* Indexing: m matvecs give H_m (m x m) and beta_m = ||f_m||, the residual uses
  beta_m; Ritz vectors y are scaled to unit 2-norm so the residual is absolute.
* Wanted set: Ritz values sorted by |mu| descending (ties: larger Im first);
  walking that list, a converged value is accepted; an unconverged value that
  lies within its own residual of any converged value or of an already accepted
  value is skipped (an unresolved copy of a multiple eigenvalue); any other
  value is accepted.  The run stops when the
  first k accepted values are all converged, at a happy breakdown
  (beta <= 64 eps ||w||) or after m matvecs.
* Inner product: Euclidean (sum over discrete unknowns), conjugating the first
  argument for complex states.

Parity status: pinned (closed-form 2x2 Schmid system, full-dimension runs against
LAPACK eig, Arnoldi-relation invariants, Ritz values within the conditioning
bound of dense eigenvalues); see tests/test_oracle_arnoldi.py.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(float).eps

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def order_ritz(mu, T):
    """Indices of Ritz values sorted by |mu| descending, ties by larger Im(lambda)
    (equivalently larger arg(mu) for T > 0)."""
    lam = np.log(mu.astype(complex)) / T
    return sorted(range(len(mu)), key=lambda i: (-abs(mu[i]), -lam[i].imag))


def select_wanted(mu, res, k, tol, T):
    """Wanted set and stop test (reading described in the module header).
    Returns (accepted indices, first-k-all-converged flag)."""
    acc = []
    conv = [i for i in range(len(mu)) if res[i] <= tol]
    for i in order_ritz(mu, T):
        if res[i] <= tol:
            acc.append(i)
        else:
            dup = any(abs(mu[i] - mu[a]) <= res[i] for a in conv + acc)
            if not dup:
                acc.append(i)
        if len(acc) >= k:
            break
    done = len(acc) >= k and all(res[a] <= tol for a in acc[:k])
    return acc[:k], done


def ritz(H, beta):
    """Ritz values, unit-norm Ritz coordinates and residual estimates |beta y_p|
    of a p x p Hessenberg matrix (LAPACK geev via numpy)."""
    mu, Y = np.linalg.eig(H)
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    res = np.abs(beta) * np.abs(Y[-1, :])
    return mu, Y, res


def arnoldi(apply, v0, m, k, tol, T=1.0, keep_basis=True):
    """Arnoldi with CGS2 on the matvec ``apply`` from start vector ``v0``.

    ``apply`` maps a 1-D array to a 1-D array of the same length.  The inner
    product is Euclidean and conjugate-linear in its first argument.
    Returns a dict with mu, lam, res (k each), X (Ritz vectors n x k), the
    accepted indices, n_matvec, status, H ((j+1) x j), beta and the basis V.
    """
    v0 = np.asarray(v0).ravel()
    n = v0.size
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= m")
    nrm0 = np.sqrt(np.vdot(v0, v0).real)
    if not np.isfinite(nrm0) or nrm0 == 0.0:
        raise ValueError("start vector must be finite and non-zero")
    v1 = v0 / nrm0
    w_first = np.asarray(apply(v1.copy())).ravel()
    # real operators on real starts stay real; anything complex is complex
    dtype = np.result_type(v0.dtype, w_first.dtype, np.float64)
    V = np.zeros((m + 1, n), dtype=dtype)
    H = np.zeros((m + 1, m), dtype=dtype)
    V[0] = v1
    status = NOT_CONVERGED
    j_done = 0
    beta = 0.0
    mu = Y = res = None
    sel = []
    for j in range(m):
        if j == 0:
            w = w_first.astype(dtype)
        else:
            w = np.asarray(apply(V[j].copy()), dtype=dtype).ravel()
        w_in = np.sqrt(np.vdot(w, w).real)
        Vj = V[: j + 1]
        h1 = Vj.conj() @ w
        w = w - Vj.T @ h1
        h2 = Vj.conj() @ w
        w = w - Vj.T @ h2
        H[: j + 1, j] = h1 + h2
        beta = np.sqrt(np.vdot(w, w).real)
        H[j + 1, j] = beta
        j_done = j + 1
        mu, Y, res = ritz(H[: j + 1, : j + 1], beta)
        breakdown = beta <= 64 * EPS * w_in
        kk = min(k, j + 1)
        sel, done = select_wanted(mu, res, kk, tol, T)
        if breakdown:
            status = BREAKDOWN
            break
        if done and kk == k:
            status = OK
            break
        V[j + 1] = w / beta
    p = j_done
    Vp = V[:p]
    Ysel = Y[:, sel]
    X = Vp.T @ Ysel
    mu_s = mu[sel]
    out = dict(
        mu=mu_s, lam=np.log(mu_s.astype(complex)) / T, res=res[sel], X=X, sel=sel,
        n_matvec=p, status=status, H=H[: p + 1, :p], beta=beta,
        all_mu=mu, all_res=res,
    )
    if keep_basis:
        out["V"] = V[: p + 1]
    return out
