"""Oracle: Krylov-Schur restarted Arnoldi on a black-box real matvec.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper, Sec. 3.2.2 ("Krylov-Schur decomposition", after Stewart 2001):
* A Krylov decomposition of order m is M V_m = V_m B_m + v_{m+1} b^T with B_m
  and b free; Arnoldi is the case B Hessenberg, b = beta e_m; Krylov-Schur the
  case B in real Schur form (1x1 and 2x2 diagonal blocks).
* The method: (1) build an m-step Arnoldi factorisation; (2) test convergence;
  (3) compute the real Schur form B = Q S Q^T ordered so that the p wanted Ritz
  values lead, giving M (V Q) = (V Q) S + v_{m+1} (b^T Q); (4) truncate to order
  p: V_p = first p columns of V Q, B = S_11, b^T = first p entries of b^T Q, and
  v_{p+1} = v_{m+1}; (5) expand back to order m with Arnoldi steps started from
  v_{p+1}, orthogonalising against every kept vector; (6) test convergence and
  return to (3) while it fails.
* Wanted Ritz values satisfy |mu| >= 1 - delta, delta typically 0.05 - 0.1.
* The residual of the Ritz pair (mu, V y) of a Krylov decomposition is
  |b^T y| (eq. "Krylov convergence"; b = beta e_m after an expansion).

Readings (where the paper leaves a choice open):
* Convergence is tested only after an expansion to order m (steps 2 and 6),
  with the wanted set and stop rule of the Arnoldi oracle (``oracle.arnoldi``):
  Ritz values by |mu| descending (ties: larger Im lambda first), unresolved
  copies of converged values skipped, stop when the first k accepted values
  have residual <= tol.
* Kept size p: the number of Ritz values with |mu| >= 1 - delta, raised to k
  and lowered to p_max (k <= p_max <= m - 2, default max(k, m // 2)); the kept
  values are the p leading ones in the order above.  When the p-th and
  (p+1)-th are the two members of a complex pair, p grows by one so the pair is
  never split (p <= m - 1, so every expansion adds at least one vector).
* Expansion steps use classical Gram-Schmidt applied twice against all
  current vectors: B[:j+1, j] = h1 + h2 and B[j+1, j] = beta_j (the last beta
  becomes b = beta e_m).  A happy breakdown (beta <= 64 eps ||w||) stops with
  exact Ritz pairs.
* At most ``max_restarts`` contractions; then NOT_CONVERGED with the Ritz pairs
  of the last B_m.
* Matvec count: m, plus m - p per restart.
* Real states only (the paper's real Schur form).

Parity status: pinned (restarted space equals the Krylov space of the
filter-polynomial start vector, the implicit-restart theorem of Sorensen 1992
and Stewart 2001; full-dimension runs against LAPACK eigenvalues; Krylov
decomposition relation and orthonormality after every restart; no restart
reduces to the Arnoldi oracle at m steps); see tests/test_oracle_krylov_schur.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from oracle.arnoldi import BREAKDOWN, NOT_CONVERGED, OK, order_ritz, select_wanted

EPS = np.finfo(float).eps


def krylov_ritz(B, b):
    """Ritz values, unit Ritz coordinates and residuals |b^T y| of the Krylov
    decomposition (B, b) (eq. "Krylov convergence"; LAPACK geev via numpy)."""
    mu, Y = np.linalg.eig(B)
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    res = np.abs(b @ Y)
    return mu, Y, res


def kept_count(mu, k, m, delta, p_max, T=1.0):
    """Number p of Ritz values kept by a restart and their indices (reading
    in the module header)."""
    order = order_ritz(mu, T)
    p = int(np.sum(np.abs(mu) >= 1.0 - delta))
    p = min(max(p, k), p_max)
    a, c = mu[order[p - 1]], mu[order[p]]
    if a.imag != 0.0 and abs(c - np.conj(a)) <= 8 * EPS * abs(a) and abs(c) == abs(a):
        p += 1
    return p, order[:p]


def cgs2_step(V, j, w):
    """Project w on the first j+1 basis vectors twice; returns (h, beta, f)."""
    Vj = V[: j + 1]
    h1 = Vj @ w
    w = w - Vj.T @ h1
    h2 = Vj @ w
    w = w - Vj.T @ h2
    return h1 + h2, np.sqrt(w @ w), w


def krylov_schur(apply, v0, m, k, tol, delta=0.1, p_max=None, max_restarts=50, T=1.0, record=None):
    """Krylov-Schur iteration (Sec. 3.2.2) on the real matvec ``apply`` from ``v0``.

    Returns a dict with mu, lam, res (k each), X (Ritz vectors n x k), sel,
    n_matvec, n_restarts, status, p_hist (kept size of every restart), B, b and
    the basis V ((m+1) x n).  ``record`` (a list or None) receives, after every
    restart, (V_p+1, B_p, b_p) for inspection by tests.
    """
    v0 = np.asarray(v0, dtype=float).ravel()
    n = v0.size
    if not (1 <= k and k + 2 <= m <= n):
        raise ValueError("need k + 2 <= m <= n")
    if p_max is None:
        p_max = max(k, m // 2)
    if not (k <= p_max <= m - 2):
        raise ValueError("need k <= p_max <= m - 2")
    nrm0 = np.sqrt(v0 @ v0)
    if not np.isfinite(nrm0) or nrm0 == 0.0:
        raise ValueError("start vector must be finite and non-zero")
    V = np.zeros((m + 1, n))
    B = np.zeros((m, m))
    b = np.zeros(m)
    V[0] = v0 / nrm0

    def expand(j0):
        """Arnoldi steps j0 .. m-1 (step 1, or step 5 after a truncation).
        Returns (matvecs done, breakdown flag)."""
        for j in range(j0, m):
            w = np.asarray(apply(V[j].copy()), dtype=float).ravel()
            w_in = np.sqrt(w @ w)
            h, beta, f = cgs2_step(V, j, w)
            B[: j + 1, j] = h
            if beta <= 64 * EPS * w_in:
                return j + 1 - j0, j + 1
            if j + 1 < m:
                B[j + 1, j] = beta
            else:
                b[:] = 0.0
                b[m - 1] = beta
            V[j + 1] = f / beta
        return m - j0, 0

    n_matvec, bd = expand(0)
    n_restarts = 0
    p_hist = []
    status = NOT_CONVERGED
    while True:
        order_m = bd if bd else m
        Bm, bm = B[:order_m, :order_m], (b if not bd else np.zeros(order_m))
        mu, Y, res = krylov_ritz(Bm, bm)
        sel, done = select_wanted(mu, res, k, tol, T)
        if bd:
            status = BREAKDOWN
            break
        if done:
            status = OK
            break
        if n_restarts >= max_restarts:
            break
        # step 3: ordered real Schur form, the p kept values leading
        p, keep = kept_count(mu, k, m, delta, p_max, T)
        kept = mu[keep]

        def wanted(re, im):
            z = re + 1j * im
            return bool(np.argmin(np.abs(mu - z)) in set(keep)) if np.all(np.isfinite(z)) else False

        S, Q, sdim = sl.schur(B, output="real", sort=wanted)
        if sdim != p:
            raise RuntimeError("Schur ordering kept %d values instead of %d" % (sdim, p))
        # step 4: truncation to order p
        Vt = Q[:, :p].T @ V[:m]
        vlast = V[m].copy()
        bt = b @ Q
        V[:p] = Vt
        V[p] = vlast
        V[p + 1:] = 0.0
        B[:] = 0.0
        B[:p, :p] = S[:p, :p]
        B[p, :p] = bt[:p]  # row p of the next B holds b_1^T (v_{p+1} = v_{m+1})
        b[:] = 0.0
        n_restarts += 1
        p_hist.append(p)
        if record is not None:
            record.append((V[: p + 1].copy(), S[:p, :p].copy(), bt[:p].copy(), np.sort_complex(kept)))
        # step 5: expansion back to order m
        mv, bd = expand(p)
        n_matvec += mv
    order_m = bd if bd else m
    X = V[:order_m].T @ Y[:, sel]
    mu_s = mu[sel]
    return dict(
        mu=mu_s, lam=np.log(mu_s.astype(complex)) / T, res=res[sel], X=X, sel=sel,
        n_matvec=n_matvec, n_restarts=n_restarts, status=status, p_hist=p_hist,
        B=B[:order_m, :order_m].copy(), b=b[:order_m].copy(), V=V.copy(), all_mu=mu, all_res=res,
    )
