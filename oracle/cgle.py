"""Oracle: linear complex Ginzburg-Landau (CGLE) operator and its Crank-Nicolson propagator.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper: Sec. 2.3.2 ("Illustration" of resolvent analysis), eq. "ginzburg-landau
equation": du/dt = -nu du/dx + gamma d2u/dx2 + mu(x) u with
mu(x) = (mu0 - c_mu^2) + mu2 x^2 / 2.  The paper defers the coefficient values
to Bagheri et al. (2009); the reading used here (also the one the HIP path uses)
is nu = U + 2 i c_u, gamma = 1 + i c_d, c_mu = c_u, time dependence e^{lambda t}.
That reading is pinned by the resolvent peak the paper prints for mu0 = 0.23
(gain close to 1000 near omega = -0.55) and by the closed-form Hermite spectrum.

Discretisation (the workload's reading): n interior nodes x_j = -L + j dx,
j = 1..n, dx = 2L/(n+1), homogeneous Dirichlet ends, second-order central
differences, Crank-Nicolson in time.  The oracle solves each implicit step with
LAPACK's banded solver (partial pivoting), which is independent of whatever
tridiagonal algorithm the HIP path uses.

Parity status: pinned (closed-form spectrum, paper's resolvent peak, exact
discrete propagator eigenvalues); see tests/test_oracle_cgle.py.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


class CGLE:
    """Discrete CGLE operator L_h (n x n, tridiagonal, complex) and M = CN(dt)^(T/dt)."""

    def __init__(self, n=256, half_width=50.0, U=2.0, c_u=0.2, c_d=-1.0,
                 mu0=0.41, mu2=-0.01, dt=0.01, T=1.0):
        self.n = int(n)
        self.L = float(half_width)
        self.dx = 2.0 * self.L / (self.n + 1)
        self.x = -self.L + self.dx * np.arange(1, self.n + 1)
        # Coefficients of the equation (Sec. 2.3.2), Bagheri-2009 reading.
        self.nu = U + 2j * c_u
        self.gamma = 1.0 + 1j * c_d
        self.mu0, self.mu2, self.c_u = mu0, mu2, c_u
        self.mu = (mu0 - c_u ** 2) + mu2 * self.x ** 2 / 2.0
        self.dt = float(dt)
        self.T = float(T)
        nsteps = self.T / self.dt
        self.nsteps = int(round(nsteps))
        if abs(nsteps - self.nsteps) > 1e-9 * max(1.0, nsteps):
            raise ValueError("T must be an integer multiple of dt")

    # ---- spatial operator -------------------------------------------------
    def bands(self):
        """(sub, main, super) diagonals of L_h: central differences of
        -nu u_x + gamma u_xx plus the local term mu(x) u."""
        dx = self.dx
        sub = self.gamma / dx ** 2 + self.nu / (2.0 * dx)
        sup = self.gamma / dx ** 2 - self.nu / (2.0 * dx)
        main = -2.0 * self.gamma / dx ** 2 + self.mu
        return sub, main, sup

    def matrix(self):
        """Dense L_h (n x n complex)."""
        sub, main, sup = self.bands()
        A = np.diag(main.astype(complex))
        A += np.diag(np.full(self.n - 1, sub), -1)
        A += np.diag(np.full(self.n - 1, sup), 1)
        return A

    def rhs(self, u):
        """L_h u (matrix-free stencil)."""
        sub, main, sup = self.bands()
        out = main * u
        out[1:] += sub * u[:-1]
        out[:-1] += sup * u[1:]
        return out

    # ---- time stepper -------------------------------------------------------
    def _lhs_banded(self):
        sub, main, sup = self.bands()
        h = 0.5 * self.dt
        ab = np.zeros((3, self.n), dtype=complex)
        ab[0, 1:] = -h * sup
        ab[1, :] = 1.0 - h * main
        ab[2, :-1] = -h * sub
        return ab

    def step(self, u):
        """One Crank-Nicolson step: (I - dt/2 L) u+ = (I + dt/2 L) u."""
        rhs = u + 0.5 * self.dt * self.rhs(u)
        return solve_banded((1, 1), self._lhs_banded(), rhs)

    def apply(self, u):
        """Matvec of the exponential propagator, M u ~ exp(L T) u, by time
        marching (Sec. 3, 'time-stepper' approach; Sec. 3.2 eq. discrete-time
        linear system)."""
        u = np.asarray(u, dtype=complex).copy()
        ab = self._lhs_banded()
        h = 0.5 * self.dt
        for _ in range(self.nsteps):
            rhs = u + h * self.rhs(u)
            u = solve_banded((1, 1), ab, rhs)
        return u

    # ---- closed forms used as pins -----------------------------------------
    def closed_form_eigs(self, count):
        """Spectrum of the continuous operator on the whole line.

        Substituting u = exp(nu x / (2 gamma)) phi turns the operator into a
        complex harmonic oscillator, so
        lambda_k = mu0 - c_u^2 - nu^2/(4 gamma) - (k + 1/2) sqrt(-2 mu2 gamma),
        principal square root.
        """
        h = np.sqrt(-2.0 * self.mu2 * self.gamma + 0j)
        k = np.arange(count)
        return (self.mu0 - self.c_u ** 2) - self.nu ** 2 / (4.0 * self.gamma) - (k + 0.5) * h

    def closed_form_mode0(self, x):
        """Leading global mode exp(nu x/(2 gamma)) exp(-chi x^2 / 2),
        chi = sqrt(-mu2 / (2 gamma)) (principal root), unnormalised."""
        chi = np.sqrt(-self.mu2 / (2.0 * self.gamma) + 0j)
        return np.exp(self.nu * x / (2.0 * self.gamma) - chi * x ** 2 / 2.0)

    def cn_propagator_eigs(self):
        """Eigenvalues of the exact discrete propagator: r(dt lambda_h)^(T/dt) with
        r(z) = (1 + z/2)/(1 - z/2), lambda_h from LAPACK on the dense L_h."""
        lam = np.linalg.eigvals(self.matrix())
        z = self.dt * lam
        return ((1 + z / 2) / (1 - z / 2)) ** self.nsteps, lam


def resolvent_gain(op: CGLE, omega):
    """Optimal resolvent gain sigma_1^2 of (i omega I - L_h)^{-1}
    (Sec. 2.3.2, definition of R(omega)).  Euclidean norm on the uniform grid is
    proportional to the L2 norm, so the gain is norm-independent."""
    A = op.matrix()
    out = []
    for w in np.atleast_1d(omega):
        s = np.linalg.svd(1j * w * np.eye(op.n) - A, compute_uv=False)
        out.append(1.0 / s[-1] ** 2)
    return np.array(out)
