"""Pins of the adjoint propagators and of the optimal-perturbation oracle
(Sec. 2.3.1 SVD formulation, Sec. 3.3.2 Lanczos on M^dagger M)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle.arnoldi import BREAKDOWN, OK, arnoldi
from oracle.cgle import CGLE
from oracle.kolmogorov import Kolmogorov, base_from_streamfunction
from oracle.optimal import (cgle_apply_adjoint, kolmo_advection_transpose, kolmo_apply_adjoint, lanczos,
                            optimal_perturbation)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _general(N, seed, dt=0.01, T=0.1, alpha=0.5, Re=20.0):
    U, V, Ox, Oy = base_from_streamfunction(W.random_base_modes(2, seed), N, alpha)
    return Kolmogorov(N, alpha, Re, dt, T, U, V, Ox, Oy)


@pytest.mark.parametrize("N,seed", [(16, 1), (32, 2)])
def test_advection_transpose_satisfies_the_dot_product_identity(N, seed):
    op = _general(N, seed)
    w = op.project(W.normal_real((N, N), seed + 10))
    z = op.project(W.normal_real((N, N), seed + 20))
    Nw = op.to_physical(op.advection_hat(op.to_spectral(w)))
    Ntz = op.to_physical(kolmo_advection_transpose(op, op.to_spectral(z)))
    lhs, rhs = np.sum(Nw * z), np.sum(w * Ntz)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Nw) * np.linalg.norm(z)
    # and the operator is not symmetric, so the identity is not vacuous
    Nz = op.to_physical(op.advection_hat(op.to_spectral(z)))
    assert abs(np.sum(Nz * w) - lhs) > 1e-3 * abs(lhs)


@pytest.mark.parametrize("kind", ["general", "kolmogorov"])
def test_adjoint_propagator_satisfies_the_dot_product_identity(kind):
    N = 32
    op = _general(N, 3) if kind == "general" else Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.01, 0.1)
    x = op.project(W.normal_real((N, N), 4))
    y = op.project(W.normal_real((N, N), 5))
    Mx, Mty = op.apply(x), kolmo_apply_adjoint(op, y)
    assert abs(np.sum(Mx * y) - np.sum(x * Mty)) <= 1e-12 * np.linalg.norm(Mx) * np.linalg.norm(y)


def test_adjoint_equals_the_dense_transpose_on_a_tiny_grid():
    N = 8
    op = _general(N, 6, dt=0.05, T=0.2)
    I = np.eye(N * N)
    M = np.stack([op.apply(I[i].reshape(N, N)).ravel() for i in range(N * N)], axis=1)
    Mt = np.stack([kolmo_apply_adjoint(op, I[i].reshape(N, N)).ravel() for i in range(N * N)], axis=1)
    assert np.max(np.abs(Mt - M.T)) <= 1e-13 * np.max(np.abs(M))
    # direct and adjoint share the spectrum (Sec. 2.2, footnote on the adjoint)
    ev, evt = np.sort_complex(np.linalg.eigvals(M)), np.sort_complex(np.linalg.eigvals(Mt))
    assert np.max(np.abs(ev - evt)) <= 1e-10


def test_cgle_adjoint_is_the_conjugate_transpose():
    op = CGLE(n=24, half_width=10.0, T=0.2)
    I = np.eye(op.n)
    M = np.stack([op.apply(I[i]) for i in range(op.n)], axis=1)
    Mh = np.stack([cgle_apply_adjoint(op, I[i]) for i in range(op.n)], axis=1)
    assert np.max(np.abs(Mh - M.conj().T)) <= 1e-13 * np.max(np.abs(M))
    x, y = W.normal_complex(op.n, 1), W.normal_complex(op.n, 2)
    assert abs(np.vdot(op.apply(x), y) - np.vdot(x, cgle_apply_adjoint(op, y))) <= 1e-12 * np.linalg.norm(x) * \
        np.linalg.norm(y) * np.max(np.abs(M))


def test_lanczos_reproduces_lapack_singular_values():
    n = 60
    B = W.random_matrix(n, 7) / np.sqrt(n) + np.diag(np.linspace(0.1, 2.0, n))
    r = optimal_perturbation(lambda v: B @ v, lambda v: B.T @ v, W.normal_real(n, 8), 60, 3, 1e-10)
    assert r["status"] == OK
    U, s, Vt = np.linalg.svd(B)
    assert np.max(np.abs(np.sort(r["sigma"])[::-1] - s[:3])) <= 1e-10 * s[0]
    for sig, x in zip(r["sigma"], r["X"].T):
        i = int(np.argmin(np.abs(s - sig)))
        assert abs(abs(Vt[i] @ x) - 1.0) <= 1e-8
        # M x = sigma u with ||u|| = 1
        assert abs(np.linalg.norm(B @ x) - sig) <= 1e-10 * s[0]


def test_lanczos_on_a_symmetric_operator_equals_arnoldi():
    n = 80
    Q, _ = np.linalg.qr(W.normal_real((n, n), 11))
    A = Q @ np.diag(np.linspace(0.0, 3.0, n)) @ Q.T
    v0 = W.normal_real(n, 12)
    lz = lanczos(lambda v: A @ v, v0, 25, 4, 0.0)
    ar = arnoldi(lambda v: A @ v, v0, 25, 4, 0.0)
    assert np.max(np.abs(np.sort(lz["all_theta"]) - np.sort(ar["all_mu"].real))) <= 1e-10
    # and the Hessenberg matrix of Arnoldi is the tridiagonal of Lanczos
    H = ar["H"][:25, :25].real
    assert np.max(np.abs(np.diag(H) - lz["alpha"])) <= 1e-12
    assert np.max(np.abs(np.diag(H, -1) - lz["beta"][:-1])) <= 1e-12
    assert np.max(np.abs(np.triu(H, 2))) <= 1e-10


def test_schmid_toy_gain_has_the_closed_form():
    g = {}
    for line in open(os.path.join(GOLD, "schmid_toy.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            g[k] = float(v)
    l1, l2, T = g["lambda1"], g["lambda2"], 10.0
    M = np.array([[np.exp(l1 * T), 0.0],
                  [(np.exp(l1 * T) - np.exp(l2 * T)) / (l1 - l2), np.exp(l2 * T)]])
    # sigma^2 are the roots of s^2 - ||M||_F^2 s + det(M)^2
    tr, det = np.sum(M * M), np.linalg.det(M)
    s1 = np.sqrt((tr + np.sqrt(tr * tr - 4 * det * det)) / 2)
    r = optimal_perturbation(lambda v: M @ v, lambda v: M.T @ v, np.array([0.3, -1.1]), 2, 1, 1e-12)
    assert r["status"] in (OK, BREAKDOWN)
    assert abs(r["sigma"][0] - s1) <= 1e-12 * s1
    assert s1 > 1.0 and max(abs(np.exp(l1 * T)), abs(np.exp(l2 * T))) < 1.0  # transient growth of a stable system


def test_kolmogorov_gain_matches_the_dense_svd():
    N = 16
    op = Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.02, 1.0)
    I = np.eye(N * N)
    P = np.stack([op.project(I[i].reshape(N, N)).ravel() for i in range(N * N)], axis=1)
    M = np.stack([op.apply(I[i].reshape(N, N)).ravel() for i in range(N * N)], axis=1) @ P
    s = np.linalg.svd(M, compute_uv=False)
    v0 = op.project(W.kolmo_start_physical(N, 0)).ravel()
    r = optimal_perturbation(lambda v: op.apply(v.reshape(N, N)).ravel(),
                             lambda v: kolmo_apply_adjoint(op, v.reshape(N, N)).ravel(), v0, 60, 3, 1e-9)
    assert r["status"] == OK
    assert abs(np.max(r["sigma"]) - s[0]) <= 1e-10 * s[0]
    for sig in r["sigma"]:
        assert np.min(np.abs(s - sig)) <= 1e-10 * s[0]


def test_cgle_gain_matches_the_dense_svd():
    op = CGLE(n=64, half_width=20.0, T=1.0)
    I = np.eye(op.n)
    M = np.stack([op.apply(I[i]) for i in range(op.n)], axis=1)
    s = np.linalg.svd(M, compute_uv=False)
    r = optimal_perturbation(op.apply, lambda v: cgle_apply_adjoint(op, v), W.normal_complex(op.n, 3), 40, 2,
                             1e-9)
    assert r["status"] == OK
    assert np.max(np.abs(np.sort(r["sigma"])[::-1] - s[:2])) <= 1e-10 * s[0]
