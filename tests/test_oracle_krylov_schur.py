"""Pins of the Krylov-Schur oracle (Sec. 3.2.2, Stewart 2001)."""
import numpy as np
import scipy.linalg as sl

from oracle.arnoldi import NOT_CONVERGED, OK, arnoldi
from oracle.kolmogorov import Kolmogorov, galerkin_sinusoidal_blocks
from oracle.krylov_schur import kept_count, krylov_schur
import workloads as W


def _filtered_krylov_space(A, v0, shifts, dim):
    """Orthonormal basis of K_dim(A, psi(A) v0), psi(z) = prod (z - shift)."""
    u = v0 / np.linalg.norm(v0)
    for t in shifts:
        u = A @ u - t * u
        u = u / np.linalg.norm(u)
    assert np.max(np.abs(u.imag)) < 1e-9  # conjugate shifts come in pairs
    K = [u.real]
    for _ in range(dim - 1):
        x = A @ K[-1]
        K.append(x / np.linalg.norm(x))
    return np.array(K).T


def test_restart_space_is_the_krylov_space_of_the_filtered_start():
    # Implicit-restart theorem (Sorensen 1992; Stewart 2001): keeping the Schur
    # vectors of the p wanted Ritz values leaves span(V_p, v_{p+1}) =
    # K_{p+1}(A, psi(A) v1), psi's roots the m - p unwanted Ritz values.
    n, m, k = 40, 12, 3
    A = W.random_matrix(n, 5) / np.sqrt(n) + np.diag(np.linspace(-1, 2, n))
    v0 = W.normal_real(n, 6)
    rec = []
    krylov_schur(lambda v: A @ v, v0, m, k, 0.0, delta=0.0, p_max=5, max_restarts=1, record=rec)
    Vp1, S, _, kept = rec[0]
    p = S.shape[0]
    assert p == 5
    theta = arnoldi(lambda v: A @ v, v0, m, m, 0.0)["all_mu"]
    unwanted = [t for t in theta if np.min(np.abs(kept - t)) > 1e-10]
    assert len(unwanted) == m - p
    K = _filtered_krylov_space(A, v0, unwanted, p + 1)
    assert np.max(sl.subspace_angles(K, Vp1.T)) < 1e-10
    assert np.max(sl.subspace_angles(K[:, :p], Vp1[:p].T)) < 1e-10


def test_krylov_decomposition_holds_after_every_restart():
    n, m, k = 120, 16, 4
    A = W.random_matrix(n, 7) / np.sqrt(n) + np.diag(np.linspace(0, 1.5, n))
    rec = []
    r = krylov_schur(lambda v: A @ v, W.normal_real(n, 8), m, k, 1e-11, delta=0.3, record=rec)
    assert r["n_restarts"] >= 2 and len(rec) == r["n_restarts"]
    nA = np.linalg.norm(A, 2)
    for Vp1, S, b1, kept in rec:
        p = S.shape[0]
        Vp, v = Vp1[:p].T, Vp1[p]
        assert np.max(np.abs(Vp1 @ Vp1.T - np.eye(p + 1))) < 1e-12
        # M V_p = V_p S_11 + v_{p+1} b_1^T
        assert np.max(np.abs(A @ Vp - Vp @ S - np.outer(v, b1))) < 1e-12 * nA
        # S_11 is in real Schur form and carries exactly the kept Ritz values
        assert np.all(np.abs(np.tril(S, -2)) == 0.0)
        sub = np.diag(S, -1)
        assert np.all((sub == 0.0)[:-1] | (sub == 0.0)[1:])  # no two adjacent 2x2 couplings
        ev = np.sort_complex(np.linalg.eigvals(S))
        assert np.max(np.abs(ev - kept)) < 1e-10 * max(1.0, np.max(np.abs(kept)))
    # the final decomposition after the last expansion: b = beta e_m
    V, B, b = r["V"], r["B"], r["b"]
    assert np.all(b[:-1] == 0.0)
    lhs = A @ V[:m].T
    rhs = V[:m].T @ B + np.outer(V[m], b)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * nA


def test_restarted_run_converges_to_lapack_eigenvalues():
    n = 200
    d = np.concatenate([[3.0, 2.5, 2.0, 1.9], np.linspace(0.1, 1.0, n - 4)])
    Q, _ = np.linalg.qr(W.normal_real((n, n), 9))
    A = Q @ np.diag(d) @ Q.T + 0.05 * W.random_matrix(n, 3) / np.sqrt(n)
    r = krylov_schur(lambda v: A @ v, W.normal_real(n, 10), 12, 4, 1e-10, delta=0.5)
    assert r["status"] == OK and r["n_restarts"] >= 1
    assert r["n_matvec"] == 12 + sum(12 - p for p in r["p_hist"])
    ev = np.linalg.eigvals(A)
    top = ev[np.argsort(-np.abs(ev))][:4]
    assert np.max(np.abs(np.sort_complex(r["mu"]) - np.sort_complex(top))) < 1e-9
    assert np.all(r["res"] <= 1e-10)
    for mu, x, res in zip(r["mu"], r["X"].T, r["res"]):
        assert abs(np.linalg.norm(A @ x - mu * x) - res) < 1e-10


def test_no_restart_reduces_to_arnoldi_after_m_steps():
    n, m, k = 80, 14, 3
    A = W.random_matrix(n, 11) / np.sqrt(n)
    v0 = W.normal_real(n, 12)
    r = krylov_schur(lambda v: A @ v, v0, m, k, 0.0, max_restarts=0)
    a = arnoldi(lambda v: A @ v, v0, m, k, 0.0)
    assert r["status"] == NOT_CONVERGED and r["n_matvec"] == m and r["n_restarts"] == 0
    assert np.max(np.abs(np.sort_complex(r["all_mu"]) - np.sort_complex(a["all_mu"]))) < 1e-12
    assert np.max(np.abs(np.sort(r["all_res"]) - np.sort(a["all_res"]))) < 1e-12


def test_kept_count_rule():
    mu = np.array([0.99, 0.97 + 0.1j, 0.97 - 0.1j, 0.95, 0.5, 0.4, 0.3, 0.2])
    # |mu| >= 0.9: four values, raised to k, lowered to p_max
    assert kept_count(mu, 2, 8, 0.1, 6)[0] == 4
    assert kept_count(mu, 5, 8, 0.1, 6)[0] == 5
    assert kept_count(mu, 2, 8, 0.6, 3)[0] == 3
    # p = 2 would split the pair (0.97 +- 0.1i): grows to 3
    p, keep = kept_count(mu, 2, 8, 0.02, 6)
    assert p == 3 and sorted(keep) == [0, 1, 2]
    # the pair's +Im member comes first
    assert list(keep)[:2] == [1, 2] or list(keep)[1:] == [1, 2]


def test_small_kolmogorov_grid_restarted_matches_dense_galerkin():
    N, alpha, Re = 16, 0.5, 20.0
    op = Kolmogorov.kolmogorov(N, alpha, Re, 0.01, 1.0)
    blocks = galerkin_sinusoidal_blocks(N, alpha, Re)
    ev = np.concatenate([np.linalg.eigvals(A) for _, A in blocks.values()])
    v0 = op.project(W.kolmo_start_physical(N, 0)).ravel()
    r = krylov_schur(lambda v: op.apply(v.reshape(N, N)).ravel(), v0, 12, 4, 1e-10, delta=0.1, T=op.T)
    assert r["status"] == OK and r["n_restarts"] >= 1
    # every converged lambda is an eigenvalue of the Galerkin operator up to the
    # time-stepping error of dt = 0.01 (fourth order)
    for lam in r["lam"]:
        assert np.min(np.abs(ev - lam)) < 1e-6
    # and the leading Galerkin eigenvalue is found
    assert np.min(np.abs(r["lam"] - ev[np.argmax(ev.real)])) < 1e-6
