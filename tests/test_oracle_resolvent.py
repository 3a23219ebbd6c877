"""Pins of the resolvent oracle (Sec. 2.3.2; Sec. 3.3.2 forced time integration)."""
import numpy as np

import workloads as W
from oracle.cgle import CGLE, resolvent_gain
from oracle.optimal import optimal_perturbation
from oracle.resolvent import discrete_resolvent, forced_response, warped_frequency


def _small():
    # a short stable domain: least stable eigenvalue about -0.4, transients die fast
    return CGLE(n=48, half_width=20.0, mu0=0.0, dt=0.01)


def test_forced_integration_reaches_the_warped_resolvent():
    op = _small()
    assert np.max(np.linalg.eigvals(op.matrix()).real) < -0.2
    f = W.normal_complex(op.n, 1)
    for omega in (-0.55, 0.3):
        got = forced_response(op, f, omega, 90.0)
        want = discrete_resolvent(op, omega) @ f
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
        # and the adjoint integration is its conjugate transpose
        g = W.normal_complex(op.n, 2)
        lhs = np.vdot(g, got)
        rhs = np.vdot(forced_response(op, g, omega, 90.0, adjoint=True), f)
        assert abs(lhs - rhs) <= 1e-9 * np.linalg.norm(got) * np.linalg.norm(g)


def test_warped_resolvent_converges_at_second_order_to_the_resolvent():
    op = _small()
    omega = -0.55
    exact = np.linalg.inv(1j * omega * np.eye(op.n) - op.matrix())
    errs = []
    for dt in (0.2, 0.1, 0.05):
        assert abs(warped_frequency(omega, dt) - omega) < 0.01
        op.dt = dt
        errs.append(np.linalg.norm(discrete_resolvent(op, omega) - exact))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.7 < errs[1] / errs[2] < 4.3


def test_lanczos_on_the_forced_integration_gives_the_resolvent_gains():
    op = _small()
    omega = -0.55
    s = np.linalg.svd(discrete_resolvent(op, omega), compute_uv=False)
    r = optimal_perturbation(lambda v: forced_response(op, v, omega, 90.0),
                             lambda v: forced_response(op, v, omega, 90.0, adjoint=True),
                             W.normal_complex(op.n, 3), 20, 2, 1e-8 * s[0] ** 2)
    assert r["status"] == 0
    assert np.max(np.abs(np.sort(r["gain"])[::-1] - s[:2] ** 2)) <= 1e-8 * s[0] ** 2
    # the leading gain equals the dense resolvent gain of L_h at the warped frequency
    assert abs(r["gain"].max() - resolvent_gain(op, warped_frequency(omega, op.dt))[0]) <= 1e-8 * s[0] ** 2
