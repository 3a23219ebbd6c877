"""Pins of the Arnoldi oracle (Sec. 3.2.1 Algorithm 1, Sec. 3.2.2 residual)."""
import os

import numpy as np
import scipy.linalg as sl

from oracle.arnoldi import BREAKDOWN, NOT_CONVERGED, OK, arnoldi, select_wanted
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_schmid_toy_breaks_down_with_exact_ritz_values():
    g = {}
    for line in open(os.path.join(GOLD, "schmid_toy.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = float(v)
    Re, T = g["Re"], 10.0
    A = np.array([[1 / 100 - 1 / Re, 0.0], [1.0, -2 / Re]])
    l1, l2 = g["lambda1"], g["lambda2"]
    # exp(A T) of a lower-triangular 2x2 in closed form
    M = np.array([[np.exp(l1 * T), 0.0],
                  [(np.exp(l1 * T) - np.exp(l2 * T)) / (l1 - l2), np.exp(l2 * T)]])
    assert np.allclose(M, sl.expm(A * T), atol=1e-14)
    r = arnoldi(lambda v: M @ v, np.array([0.3, -1.1]), 5, 2, 1e-12, T=T)
    assert r["status"] == BREAKDOWN and r["n_matvec"] == 2
    assert np.allclose(np.sort(r["lam"].real), [l2, l1], atol=1e-13)


def test_full_dimension_run_reproduces_lapack_eigenvalues():
    for cplx in (False, True):
        A = W.random_matrix(24, 1, complex_=cplx) / 5.0
        v0 = W.normal_real(24, 2)
        r = arnoldi(lambda v: A @ v, v0, 24, 24, 0.0)
        ev = np.linalg.eigvals(A)
        for mu in r["all_mu"]:
            assert np.min(np.abs(ev - mu)) < 1e-10 * np.max(np.abs(ev))


def test_arnoldi_relation_orthogonality_and_residual_identity():
    n, m = 300, 40
    A = W.random_matrix(n, 3) / np.sqrt(n) + np.diag(np.linspace(0, 2, n))
    r = arnoldi(lambda v: A @ v, W.normal_real(n, 4), m, 6, 0.0)
    V, H = r["V"], r["H"]
    assert r["status"] == NOT_CONVERGED and r["n_matvec"] == m
    assert np.max(np.abs(V @ V.T - np.eye(m + 1))) < 1e-13
    lhs = A @ V[:m].T
    rhs = V[:m].T @ H[:m] + np.outer(V[m], H[m])
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.linalg.norm(A, 2)
    # |beta e_m^T y| equals ||A x - mu x|| for unit y (eq. Krylov convergence)
    for mu, x, res in zip(r["mu"], r["X"].T, r["res"]):
        true = np.linalg.norm(A @ x - mu * x)
        assert abs(true - res) <= 1e-10 * max(1.0, res) + 1e-12


def test_wanted_set_skips_unresolved_copies_and_stops():
    mu = np.array([0.9, 0.9 + 1e-9, 0.5, 0.4])
    res = np.array([1e-10, 1e-6, 1e-10, 1e-3])
    sel, done = select_wanted(mu, res, 2, 1e-8, 1.0)
    assert sel == [0, 2] and done
    sel, done = select_wanted(mu, res, 3, 1e-8, 1.0)
    assert sel == [0, 2, 3] and not done
    # an unconverged value far from every accepted one blocks convergence
    res2 = np.array([1e-10, 1e-12, 1e-10, 1e-3])
    sel, done = select_wanted(mu, res2, 3, 1e-8, 1.0)
    assert sel == [1, 0, 2] or sel == [0, 1, 2]
    assert done


def test_stops_as_soon_as_k_wanted_pairs_converge():
    n = 200
    d = np.concatenate([[3.0, 2.5, 2.0], np.linspace(0.1, 1.0, n - 3)])
    Q, _ = np.linalg.qr(W.normal_real((n, n), 9))
    A = Q @ np.diag(d) @ Q.T
    r = arnoldi(lambda v: A @ v, W.normal_real(n, 10), 60, 3, 1e-8)
    assert r["status"] == OK
    assert np.allclose(np.sort(r["mu"].real), [2.0, 2.5, 3.0], atol=1e-9)
    assert np.all(r["res"] <= 1e-8)
    # one step fewer would not have converged
    r2 = arnoldi(lambda v: A @ v, W.normal_real(n, 10), r["n_matvec"] - 1, 3, 1e-8)
    assert r2["status"] == NOT_CONVERGED
