"""Pins of the Kolmogorov / linearized Navier-Stokes oracle (Sec. 3) against
independent constructions.  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle.arnoldi import BREAKDOWN, arnoldi
from oracle.kolmogorov import (Kolmogorov, base_from_streamfunction, base_vorticity_gradient,
                               brute_force_advection, dealias_cutoff,
                               galerkin_sinusoidal_advection, galerkin_sinusoidal_blocks)
import workloads as W


def _rand_hat(op, seed):
    return op.to_spectral(W.normal_real((op.N, op.N), seed))


@pytest.mark.parametrize("N,n_forcing,alpha", [(16, 4, 0.5), (24, 4, 1.0), (32, 2, 0.75)])
def test_grid_products_equal_closed_form_coupling(N, n_forcing, alpha):
    op = Kolmogorov.kolmogorov(N, alpha, 20.0, 0.005, 1.0, n_forcing=n_forcing)
    wh = _rand_hat(op, 1)
    a = op.advection_hat(wh)
    b = galerkin_sinusoidal_advection(op, wh, n_forcing)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("seed", [3, 4])
def test_grid_products_equal_brute_force_convolution_general_base(seed):
    N, alpha = 16, 0.5
    modes = W.random_base_modes(2, seed)
    U, V, Ox, Oy = base_from_streamfunction(modes, N, alpha)
    op = Kolmogorov(N, alpha, 20.0, 0.005, 1.0, U, V, Ox, Oy)
    wh = _rand_hat(op, seed + 10)
    a = op.advection_hat(wh)
    b = brute_force_advection(op, wh, modes)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_reflection_symmetry_ties_cross_terms():
    # Swapping x and y (square box) maps the base (U, V, Ox, Oy) to
    # (V^T, U^T, -Oy^T, -Ox^T) and commutes with the linearized advection.
    N = 16
    modes = W.random_base_modes(2, 7)
    U, V, Ox, Oy = base_from_streamfunction(modes, N, 1.0)
    op = Kolmogorov(N, 1.0, 20.0, 0.005, 1.0, U, V, Ox, Oy)
    opT = Kolmogorov(N, 1.0, 20.0, 0.005, 1.0, V.T, U.T, -Oy.T, -Ox.T)
    w = op.project(W.normal_real((N, N), 8))
    a = op.to_physical(op.advection_hat(op.to_spectral(w)))
    b = opT.to_physical(opT.advection_hat(opT.to_spectral(w.T)))
    assert np.max(np.abs(a.T - b)) <= 1e-12 * np.max(np.abs(a))
    # and the symmetry is not trivially satisfied by a base without cross terms
    assert np.max(np.abs(V)) > 0.1 and np.max(np.abs(Ox)) > 0.1


def test_base_vorticity_gradient_spectral_matches_analytic():
    N, alpha = 24, 0.5
    modes = W.random_base_modes(3, 5)
    U, V, Ox, Oy = base_from_streamfunction(modes, N, alpha)
    gx, gy = base_vorticity_gradient(U, V, alpha)
    assert np.max(np.abs(gx - Ox)) < 1e-11 and np.max(np.abs(gy - Oy)) < 1e-11


def test_if_rk4_is_fourth_order_against_matrix_exponential():
    # Lawson RK4 on a kx column (a closed linear subsystem) converges to
    # expm(A T) of the dense Galerkin block at fourth order.
    N, alpha, Re, T = 16, 0.5, 20.0, 0.4
    jx = 2
    blocks = galerkin_sinusoidal_blocks(N, alpha, Re)
    jys, A = blocks[jx]
    rng = np.random.default_rng(0)
    c0 = rng.standard_normal(len(jys)) + 1j * rng.standard_normal(len(jys))
    ref = sl.expm(A * T) @ c0
    errs = []
    for dt in (0.1, 0.05, 0.025):
        op = Kolmogorov.kolmogorov(N, alpha, Re, dt, T)
        wh = np.zeros((N, N // 2 + 1), complex)
        for c, j in zip(c0, jys):
            wh[j % N, jx] = c
        for _ in range(op.nsteps):
            wh = op.step_hat(wh)
        got = np.array([wh[j % N, jx] for j in jys])
        errs.append(np.linalg.norm(got - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r1 < 19 and 13 < r2 < 19, errs


def test_arnoldi_on_stepper_matches_dense_galerkin_eigenvalues():
    N, alpha, Re = 32, 0.5, 20.0
    op = Kolmogorov.kolmogorov(N, alpha, Re, 0.005, 1.0)
    blocks = galerkin_sinusoidal_blocks(N, alpha, Re)
    ev = np.concatenate([np.linalg.eigvals(A) for _, A in blocks.values()])
    lead = np.sort(ev.real)[::-1]
    lead = lead[np.concatenate([[True], np.diff(lead) < -1e-9])][:5]
    v0 = op.project(W.kolmo_start_physical(N, 0)).ravel()
    r = arnoldi(lambda v: op.apply(v.reshape(N, N)).ravel(), v0, 60, 5, 1e-10, T=op.T)
    assert r["status"] == 0
    got = np.sort(r["lam"].real)[::-1]
    assert np.max(np.abs(got - lead)) < 1e-8
    assert np.max(np.abs(r["lam"].imag)) < 1e-10


def test_exact_eigenvector_start_breaks_down_after_one_matvec():
    N, Re = 32, 20.0
    op = Kolmogorov.kolmogorov(N, 0.5, Re, 0.005, 1.0)
    x, y = op.grid()
    w = np.repeat(np.cos(3 * y)[:, None], N, axis=1)
    r = arnoldi(lambda v: op.apply(v.reshape(N, N)).ravel(), w.ravel(), 10, 1, 1e-10, T=op.T)
    assert r["status"] == BREAKDOWN and r["n_matvec"] == 1
    assert abs(r["mu"][0] - np.exp(-9 * op.T / Re)) < 1e-13


def test_dealias_cutoff_values():
    assert [dealias_cutoff(n) for n in (128, 256, 384, 512)] == [42, 85, 127, 170]
