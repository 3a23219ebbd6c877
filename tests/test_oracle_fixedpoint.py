"""Pins of the nonlinear stepper and of the fixed-point solvers (Sec. 3.1)."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle.fixedpoint import NonlinearKolmogorov, boostconv, rpm, sfd, sfd_coupling, sfd_step, unstable_basis


def test_dealiased_advection_conserves_energy_and_enstrophy():
    # the 2/3-rule truncation of the quadratic term is an exact Galerkin
    # projection, so <N(w), w> = 0 (enstrophy) and <N(w), psi> = 0 (energy)
    for N in (16, 32):
        op = NonlinearKolmogorov(N, 0.5, 20.0, 0.01, 0.1)
        L = op.lin
        wh = L.to_spectral(W.normal_real((N, N), N))
        nh = op.advection_hat(wh)
        n, w = L.to_physical(nh), L.to_physical(wh)
        psi = L.to_physical(wh * L.invK2)
        scale = np.linalg.norm(n) * np.linalg.norm(w)
        assert abs(np.sum(n * w)) <= 1e-13 * scale
        assert abs(np.sum(n * psi)) <= 1e-13 * np.linalg.norm(n) * np.linalg.norm(psi)
        assert np.linalg.norm(n) > 1e-3 * np.linalg.norm(w)  # not vacuous


@pytest.mark.parametrize("U0", [0.0, 0.7])
def test_laminar_kolmogorov_flow_is_a_fixed_point(U0):
    op = NonlinearKolmogorov(32, 0.5, 20.0, 0.005, 1.0, U0=U0)
    w = op.omega_lam
    assert np.max(np.abs(op.apply(w) - w)) <= 1e-13 * np.max(np.abs(w))


@pytest.mark.parametrize("U0", [0.0, 0.7])
def test_jacobian_of_the_nonlinear_stepper_is_the_linearized_propagator(U0):
    N = 16
    op = NonlinearKolmogorov(N, 0.5, 20.0, 0.02, 0.4, U0=U0)
    lin = op.linearized()
    v = lin.project(W.normal_real((N, N), 3))
    v /= np.linalg.norm(v)
    eps = 1e-5
    fd = (op.apply(op.omega_lam + eps * v) - op.apply(op.omega_lam - eps * v)) / (2 * eps)
    Mv = lin.apply(v)
    assert np.linalg.norm(fd - Mv) <= 1e-8 * np.linalg.norm(Mv)


def _linear_map(n, seed):
    """G(x) = M x + b with two unstable eigenvalues (a complex pair) and a real one."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = np.diag(np.concatenate([[1.3], np.linspace(-0.8, 0.8, n - 1)]))
    D[1, 2], D[2, 1] = 0.6, -0.6  # eigenvalues 0.0... +- 0.6i block
    D[1, 1] = D[2, 2] = 0.9       # |mu| = 1.08, oscillating
    M = Q @ D @ Q.T
    b = rng.standard_normal(n)
    return M, b, np.linalg.solve(np.eye(n) - M, b)


def test_plain_iteration_diverges_and_rpm_converges_on_a_linear_map():
    M, b, xs = _linear_map(40, 1)
    G = lambda x: M @ x + b
    x = np.zeros(40)
    for _ in range(60):
        x = G(x)
    assert np.linalg.norm(x - xs) > 1e3
    U, H, kept = unstable_basis(lambda v: M @ v, W.normal_real(40, 2), 40, 1, 0.0)
    assert U.shape[1] == 3 and np.all(np.abs(kept) >= 1.0)
    xr, hist, it = rpm(G, np.zeros(40), U, H, 1e-12, 200)
    assert np.linalg.norm(xr - xs) <= 1e-11 * np.linalg.norm(xs)
    assert it < 200


def test_boostconv_converges_on_a_linear_map():
    M, b, xs = _linear_map(40, 3)
    x, hist, it = boostconv(lambda v: M @ v + b, np.zeros(40), 10, 1e-12, 400)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert it < 400


def test_sfd_coupling_is_the_exact_exponential_and_damps_an_oscillating_instability():
    chi, delta, h = 0.3, 2.0, 0.01
    E = sfd_coupling(chi, delta, h)
    # the coupling conserves X - Y's decay rate and the weighted mean (X + chi Delta Y)
    B = np.array([[-chi, chi], [1 / delta, -1 / delta]])
    assert np.allclose(E, sl.expm(h * B), atol=1e-15)
    w = np.array([1.0, chi * delta])
    assert np.allclose(w @ E, w, atol=1e-15)
    # x' = A x + b with an unstable oscillating pair: SFD reaches -A^-1 b
    A = np.array([[0.1, 1.0], [-1.0, 0.1]])
    bb = np.array([0.5, -0.2])
    xs = -np.linalg.solve(A, bb)
    step = lambda x: sl.expm(h * A) @ x + np.linalg.solve(A, (sl.expm(h * A) - np.eye(2)) @ bb)
    x, hist, steps = sfd(step, np.zeros(2), 0.5, 1.0, h, 100, 1e-10, 2000)
    assert np.linalg.norm(x - xs) <= 1e-9
    # and it cannot quench a real unstable eigenvalue: the run does not converge
    A2 = np.array([[0.1, 0.0], [0.0, -1.0]])
    xs2 = -np.linalg.solve(A2, bb)
    step2 = lambda x: sl.expm(h * A2) @ x + np.linalg.solve(A2, (sl.expm(h * A2) - np.eye(2)) @ bb)
    x2, hist2, _ = sfd(step2, xs2 + 1e-3, 0.5, 1.0, h, 100, 1e-10, 300)
    assert np.linalg.norm(x2 - xs2) > 1.0


def test_sfd_splitting_is_second_order_in_the_time_step():
    # against the exact solution of the linear extended system
    # [X; Y]' = [[A - chi, chi], [1/Delta, -1/Delta]] [X; Y]
    A = np.array([[0.1, 1.0], [-1.0, 0.1]])
    chi, delta, t = 0.5, 1.0, 2.0
    B = np.block([[A - chi * np.eye(2), chi * np.eye(2)], [np.eye(2) / delta, -np.eye(2) / delta]])
    z0 = np.array([1.0, -0.5, 1.0, -0.5])
    exact = sl.expm(t * B) @ z0
    errs = []
    for h in (0.1, 0.05, 0.025):
        E = sfd_coupling(chi, delta, 0.5 * h)
        S = sl.expm(h * A)
        X, Y = z0[:2].copy(), z0[2:].copy()
        for _ in range(int(round(t / h))):
            X, Y = sfd_step(lambda v: S @ v, E, X, Y)
        errs.append(np.linalg.norm(np.concatenate([X, Y]) - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def _forced_problem(N=16, dt=0.02, T=2.0):
    """Re = 7, drift 0.7, a weak two-dimensional extra forcing: three weakly
    unstable travelling modes about a two-dimensional fixed point."""
    ex = W.random_forcing_field(N, 0.5, 2, 7, 0.002)
    return NonlinearKolmogorov(N, 0.5, 7.0, dt, T, U0=0.7, extra_forcing=ex)


def test_fields_of_a_state_give_the_linearized_right_hand_side_about_it():
    # the advection is quadratic, so a central difference of the nonlinear
    # right-hand side about a two-dimensional state w is exactly (to rounding)
    # the linearized operator with w's own fields as base flow
    N = 16
    op = NonlinearKolmogorov(N, 0.5, 7.0, 0.02, 0.4, U0=0.7, extra_forcing=W.random_forcing_field(N, 0.5, 2, 3, 0.1))
    w = op.omega_lam + op.lin.project(W.random_forcing_field(N, 0.5, 2, 4, 0.3))
    lin = op.linearized_about(w)
    L = op.lin
    wh = L.to_spectral(w)
    vh = L.to_spectral(W.normal_real((N, N), 5))
    eps = 1e-2
    fd = (op.rhs_nl_hat(wh + eps * vh) - op.rhs_nl_hat(wh - eps * vh)) / (2 * eps)
    an = lin.advection_hat(vh)
    assert np.linalg.norm(fd - an) <= 1e-12 * np.linalg.norm(an)


def test_solvers_reach_the_same_two_dimensional_fixed_point():
    N = 16
    op = _forced_problem(N)
    G = lambda v: op.apply(v.reshape(N, N)).ravel()
    x0 = op.omega_lam.ravel().copy()
    # plain time marching leaves the (unstable) fixed point's neighbourhood
    x, hp = x0.copy(), []
    for _ in range(20):
        xn = G(x)
        hp.append(np.linalg.norm(xn - x))
        x = xn
    assert hp[-1] > hp[0]
    lin = op.linearized_about(x0.reshape(N, N))
    r0 = G(x0) - x0
    U, H, kept = unstable_basis(lambda v: lin.apply(v.reshape(N, N)).ravel(), r0, 24, 1, 0.3)
    assert np.sum(np.abs(kept) > 1.0) == 6  # three travelling modes, each a conjugate pair
    xr, hist, it = rpm(G, x0, U, H, 1e-8, 60)
    assert hist[-1] <= 1e-8
    xb, hb, itb = boostconv(G, x0, 10, 1e-9, 60)
    assert hb[-1] <= 1e-9
    assert np.linalg.norm(xr - xb) <= 1e-6
    # the fixed point is two-dimensional: it is not the laminar flow
    assert np.linalg.norm(xb - x0) > 1e-3 * np.linalg.norm(x0)
