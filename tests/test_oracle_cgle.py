"""Pins of the CGLE oracle against closed forms and the paper's printed resolvent
peak (Sec. 2.3.2).  CPU only."""
import os

import numpy as np
import pytest

from oracle.arnoldi import arnoldi
from oracle.cgle import CGLE, resolvent_gain
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    from conftest import golden
    return golden(name)


def _leading(lams, count):
    return lams[np.argsort(-lams.real)][:count]


def test_fd_spectrum_converges_to_hermite_closed_form_at_second_order():
    # Dense eig of the FD operator tends to the closed-form global-mode spectrum
    # lambda_k = mu0 - c_u^2 - nu^2/(4 gamma) - (k+1/2) sqrt(-2 mu2 gamma).
    errs = []
    for n in (256, 512, 1024):
        op = CGLE(n=n)
        lam_h = _leading(np.linalg.eigvals(op.matrix()), 4)
        ex = op.closed_form_eigs(4)
        errs.append(np.abs(lam_h - ex))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.8) and np.all(ratios < 4.2), ratios
    assert errs[-1, 0] < 1e-3


def test_closed_form_values():
    # Spot values of the closed form (arithmetic on the formula, a guard against
    # editing the coefficient reading by accident).
    ex = CGLE().closed_form_eigs(2)
    assert abs(ex[0] - (0.0123113013 - 0.6478202874j)) < 1e-9
    assert abs(ex[1] - (-0.1430660961 - 0.5834608621j)) < 1e-9


def test_leading_mode_shape_matches_closed_form():
    # The advection sign and coefficient reading are fixed by the shape of the
    # leading global mode exp(nu x / 2 gamma) exp(-chi x^2/2): it peaks downstream.
    op = CGLE(n=1024)
    lam, vec = np.linalg.eig(op.matrix())
    i = np.argmax(lam.real)
    v = vec[:, i]
    ref = op.closed_form_mode0(op.x)
    v = v / v[np.argmax(np.abs(v))]
    ref = ref / ref[np.argmax(np.abs(v))]
    assert op.x[np.argmax(np.abs(v))] > 3.0
    assert np.linalg.norm(v - ref) / np.linalg.norm(ref) < 2e-2


def test_resolvent_peak_matches_paper():
    g = _golden("cgle_resolvent_peak.txt")
    op = CGLE(n=400, half_width=85.0, mu0=0.23)
    omegas = np.arange(-0.65, -0.449, 0.01)
    gains = resolvent_gain(op, omegas)
    i = int(np.argmax(gains))
    assert abs(omegas[i] - g["omega_peak"]) <= g["omega_window"]
    assert g["gain_lower"] < gains[i] < g["gain_upper"]
    # The paper states the mu0 = 0.23 model is linearly stable.
    assert np.max(np.linalg.eigvals(op.matrix()).real) < 0


def test_propagator_acts_as_rational_function_on_eigenvectors():
    # apply() (time marching with a banded solver) on a dense-eig eigenvector
    # multiplies it by r(dt lambda)^(T/dt), r(z) = (1+z/2)/(1-z/2).
    op = CGLE()
    lam, vec = np.linalg.eig(op.matrix())
    for i in np.argsort(-lam.real)[:4]:
        v = vec[:, i]
        z = op.dt * lam[i]
        mu = ((1 + z / 2) / (1 - z / 2)) ** op.nsteps
        w = op.apply(v)
        assert np.linalg.norm(w - mu * v) <= 1e-11 * np.linalg.norm(w)


def test_arnoldi_ritz_values_within_conditioning_bound():
    # Ritz values from Arnoldi on the time stepper agree with the exact discrete
    # propagator eigenvalues to within kappa_i * residual_i (kappa from left and
    # right dense eigenvectors), the bound of first-order perturbation theory.
    c = W.CGLE
    op = CGLE()
    r = arnoldi(op.apply, W.cgle_start(256, 0), c["m"], c["k"], c["tol"], T=op.T)
    assert r["status"] == 0
    mu_ex, lam = op.cn_propagator_eigs()
    A = op.matrix()
    wl, VL, VR = None, None, None
    import scipy.linalg as sl
    w_, VL, VR = sl.eig(A, left=True, right=True)
    z = op.dt * w_
    mu_all = ((1 + z / 2) / (1 - z / 2)) ** op.nsteps
    for m_r, res in zip(r["mu"], r["res"]):
        i = np.argmin(np.abs(mu_all - m_r))
        kappa = np.linalg.norm(VL[:, i]) * np.linalg.norm(VR[:, i]) / abs(np.vdot(VL[:, i], VR[:, i]))
        assert abs(mu_all[i] - m_r) <= 2 * kappa * res + 1e-13
    # The three best-conditioned leading modes are accurate to 1e-9 outright.
    lead = np.sort(np.abs(mu_all))[::-1][:3]
    assert np.allclose(np.sort(np.abs(r["mu"]))[::-1][:3], lead, atol=1e-9)
