"""Oracle: resolvent analysis by forced time integration (Ginzburg-Landau).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper:
* Sec. 2.3.2 ("Resolvent analysis"): for the forced stable system
  x' = A x + f with harmonic forcing, the asymptotic response at frequency omega
  is x^ = R(omega) f^, R(omega) = (i omega I - A)^-1; the optimal gain is
  sigma_1^2 of R(omega), the optimal forcing and response are the leading right
  and left singular vectors.  Illustration: the linear Ginzburg-Landau equation
  with mu0 = 0.23 (stable), gain close to 1000 near omega = -0.55.
* Sec. 3.3.2: R(omega) f^ is computed by integrating the forced system forward in
  time and taking the Fourier transform of the asymptotic response; R^dagger by
  the adjoint system; the singular values by Lanczos on R^dagger R
  (``oracle.optimal``).

Readings:
* The forcing is complex, f(t) = f^ e^{i omega t} (the complex Ginzburg-Landau
  state is complex), integrated from rest with Crank-Nicolson and the trapezoidal
  rule for the forcing: (I - dt/2 L) u+ = (I + dt/2 L) u + dt/2 (f(t_n) + f(t_{n+1})).
  The asymptotic response is a single harmonic, so its Fourier coefficient over
  any window is u(t) e^{-i omega t}; it is read after t_trans time units, when
  the transient has decayed (decay rate: the least stable eigenvalue).
* The discrete periodic response of Crank-Nicolson is exactly the resolvent of
  L_h at the warped frequency w~ = (2/dt) tan(omega dt/2), (i w~ I - L_h)^-1 f^,
  which tends to R(omega) f^ at second order in dt.
* R^dagger = (-i w~ I - L_h^H)^-1: the same forced integration with L_h^H at
  frequency -omega, so R^dagger R is Hermitian to the transient remainder and the
  Lanczos iteration of ``oracle.optimal`` applies.

Parity status: pinned (the forced integration against the closed-form warped
resolvent of the discrete operator; second-order convergence of the warped
resolvent to (i omega - L_h)^-1; Lanczos on R^dagger R against the dense SVD;
the paper's printed gain peak through ``tests/test_oracle_cgle.py``); see
tests/test_oracle_resolvent.py.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def _bands(op, adjoint):
    sub, main, sup = op.bands()
    if adjoint:
        return np.conj(sup), np.conj(main), np.conj(sub)
    return sub, main, sup


def forced_response(op, f, omega, t_trans, adjoint=False):
    """u(t) e^{-i w t} after integrating u' = L u + f e^{i w t} from u = 0 over
    t_trans (Crank-Nicolson, trapezoidal forcing).  adjoint: L^H and -omega."""
    sub, main, sup = _bands(op, adjoint)
    w = -omega if adjoint else omega
    h = 0.5 * op.dt
    nsteps = int(round(t_trans / op.dt))
    ab = np.zeros((3, op.n), dtype=complex)
    ab[0, 1:] = -h * sup
    ab[1, :] = 1.0 - h * main
    ab[2, :-1] = -h * sub
    f = np.asarray(f, dtype=complex)
    c1 = h * (1.0 + np.exp(1j * w * op.dt))
    u = np.zeros(op.n, dtype=complex)
    for s in range(nsteps):
        r = main * u
        r[1:] += sub * u[:-1]
        r[:-1] += sup * u[1:]
        rhs = u + h * r + c1 * np.exp(1j * w * s * op.dt) * f
        u = solve_banded((1, 1), ab, rhs)
    return u * np.exp(-1j * w * nsteps * op.dt)


def warped_frequency(omega, dt):
    """The frequency at which Crank-Nicolson's periodic response is the exact
    resolvent of L_h: (e^{i w dt} - 1)/(dt/2 (e^{i w dt} + 1)) = i (2/dt) tan(w dt/2)."""
    return 2.0 / dt * np.tan(omega * dt / 2.0)


def discrete_resolvent(op, omega):
    """(i w~ I - L_h)^-1 as a dense matrix (the closed form of the forced
    Crank-Nicolson response)."""
    wt = warped_frequency(omega, op.dt)
    return np.linalg.inv(1j * wt * np.eye(op.n) - op.matrix())
