"""Oracle: nonlinear forced Navier-Stokes time-stepper and the fixed-point solvers
that run on it (selective frequency damping, recursive projection method,
BoostConv).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper:
* Sec. 3.1: a fixed point solves F(X) = 0 (continuous time) or X - G(X) = 0
  (discrete time, G the nonlinear time-stepper over T).
* Sec. 3.1.1, selective frequency damping (Akervik et al. 2006): the extended
  system dX/dt = F(X) - chi (X - Y), dY/dt = (X - Y)/Delta, exponential filter
  of cutoff omega_c = 1/Delta; it cannot quench non-oscillating instabilities.
* Sec. 3.1.2, recursive projection method (Shroff & Keller 1993): with U an
  orthonormal basis of the unstable invariant subspace of the Jacobian
  M = exp(A T) and H = U^T M U, the iterate is
  x~_{k+1} = x_{k+1} - U U^T (x_{k+1} - x~_k) + U (I - H)^-1 U^T (x_{k+1} - x~_k),
  x_{k+1} = G(x~_k); U from the Arnoldi or Krylov-Schur decompositions of M.
* Sec. 3.1.3, BoostConv (Citro et al. 2017): with X the corrected residuals and
  Y the residual decrements of the last iterations,
  x~_{k+1} = x_{k+1} - Y Y^+ (x_{k+1} - x~_k) + X Y^+ (x_{k+1} - x~_k).
* Sec. 3 (linearized Navier-Stokes): the nonlinear equation in vorticity form is
  d omega/dt + u . grad omega = Re^-1 lap omega + f, whose linearization about a
  base flow is the operator of ``oracle.kolmogorov``.

Readings (where the paper leaves a choice open):
* Nonlinear stepper: the same discretisation as the linearized one (N x N grid,
  2/3 rule, mean mode removed, Lawson IF-RK4), the advection (u + U0) d_x omega +
  v d_y omega of the total vorticity with u = d_y psi, v = -d_x psi, -lap psi =
  omega, an optional uniform drift U0 along x, and the steady forcing
  f = -Re^-1 lap omega_lam that holds the laminar Kolmogorov flow
  omega_lam = -n cos(n y) steady, plus an optional extra forcing field.  The
  laminar flow is then a fixed point of the discrete stepper up to the O(h^4)
  steady-state error of the Lawson scheme.  The drift makes the Kolmogorov
  instability travel (oscillating), the case selective frequency damping can
  quench.  The extra forcing breaks the x-translation symmetry, whose double
  eigenvalues a single Krylov sequence resolves along one direction only, and
  makes the fixed point two-dimensional with no analytic form.
* Jacobian for RPM: the linearized operator about a state w has w's own fields
  as its base flow (u + U0, v from w's streamfunction, grad w).
* SFD: encapsulated splitting (Jordi et al. 2014, cited in Sec. 3.1.1), Strang
  form: each time step is the exact solution over dt/2 of the linear coupling
  X' = -chi (X - Y), Y' = (X - Y)/Delta, one step of size dt of the original
  system, and the coupling over dt/2 again (second order in dt).
* RPM: U and H = U^T M U from the Krylov-Schur contraction of an Arnoldi
  factorisation of the Jacobian about the initial iterate (kept set: |mu| >=
  1 - delta), started from the initial residual G(x0) - x0 and computed once
  before the iterations; I - H is solved densely.
* BoostConv: X holds the applied corrections xi_j = x~_{j+1} - x~_j, Y the
  residual decrements r_j - r_{j+1}, r_j = G(x~_j) - x~_j, for the last m
  iterations; c = Y^+ r, the minimum-norm least-squares solution (the
  pseudo-inverse of Sec. 3.1.3), by an SVD-based least-squares solve.
* Convergence: ||r_k|| <= tol (the residual of the discrete-time fixed point,
  Euclidean state norm).

Parity status: pinned (the dealiased nonlinear term conserves energy and
enstrophy exactly; the laminar flow is a fixed point; the finite-difference
Jacobian of the nonlinear stepper equals the linearized oracle's propagator; the
solvers reach the exact fixed point of linear maps, (I - M)^-1 b, and the laminar
flow of the nonlinear stepper); see tests/test_oracle_fixedpoint.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from oracle.kolmogorov import Kolmogorov


class NonlinearKolmogorov:
    """Forced 2-D Navier-Stokes in vorticity form on the grid of ``Kolmogorov``."""

    def __init__(self, N, alpha, Re, dt, T, n_forcing=4, U0=0.0, extra_forcing=None):
        self.lin = Kolmogorov.kolmogorov(N, alpha, Re, dt, T, n_forcing)  # grid, masks, transforms
        self.N, self.alpha, self.Re, self.dt, self.T = N, float(alpha), float(Re), float(dt), float(T)
        self.nsteps = self.lin.nsteps
        self.U0 = float(U0)
        x, y = self.lin.grid()
        self.omega_lam = np.repeat((-n_forcing * np.cos(n_forcing * y))[:, None], N, axis=1)
        L = self.lin
        # -Re^-1 lap omega_lam holds the laminar flow steady; an extra forcing
        # field (physical, projected) makes the steady state two-dimensional
        self.f_hat = (L.K2 / self.Re) * L.to_spectral(self.omega_lam)
        if extra_forcing is not None:
            self.f_hat = self.f_hat + L.to_spectral(extra_forcing)

    def fields(self, w):
        """Grid fields (u + U0, v, omega_x, omega_y) of the vorticity w (physical):
        the velocity and vorticity gradient of w as a base flow."""
        L = self.lin
        irf = lambda f: np.fft.irfft2(f, s=(self.N, self.N))
        wh = L.to_spectral(w)
        psih = wh * L.invK2
        return (irf(1j * L.ky * psih) + self.U0, irf(-1j * L.kx * psih), irf(1j * L.kx * wh), irf(1j * L.ky * wh))

    def advection_hat(self, wh):
        """-P((u + U0) omega_x + v omega_y), products on the grid."""
        L = self.lin
        irf = lambda f: np.fft.irfft2(f, s=(self.N, self.N))
        psih = wh * L.invK2
        wx, wy = irf(1j * L.kx * wh), irf(1j * L.ky * wh)
        u, v = irf(1j * L.ky * psih), irf(-1j * L.kx * psih)
        return -np.fft.rfft2((u + self.U0) * wx + v * wy) * L.mask

    def rhs_nl_hat(self, wh):
        """Advection plus forcing (the part the Lawson scheme treats explicitly)."""
        return self.advection_hat(wh) + self.f_hat

    def step_hat(self, wh, h=None):
        """One Lawson IF-RK4 step (the scheme of ``Kolmogorov.step_hat``)."""
        L = self.lin
        h = self.dt if h is None else h
        E1 = np.exp(-L.K2 * h / self.Re)
        Eh = np.exp(-L.K2 * (h / 2) / self.Re)
        Nf = self.rhs_nl_hat
        a = Nf(wh)
        b = Nf(Eh * (wh + (h / 2) * a))
        c = Nf(Eh * wh + (h / 2) * b)
        d = Nf(E1 * wh + h * Eh * c)
        return E1 * wh + (h / 6) * (E1 * a + 2 * Eh * (b + c) + d)

    def apply(self, w, nsteps=None):
        """G(w): march the nonlinear equation over T (physical field in and out)."""
        wh = self.lin.to_spectral(w)
        for _ in range(self.nsteps if nsteps is None else nsteps):
            wh = self.step_hat(wh)
        return self.lin.to_physical(wh)

    def linearized_about(self, w):
        """The linearized operator (Jacobian of the right-hand side) about the
        state w: ``Kolmogorov`` with w's fields as the base flow."""
        U, V, Ox, Oy = self.fields(w)
        return Kolmogorov(self.N, self.alpha, self.Re, self.dt, self.T, U, V, Ox, Oy)

    def linearized(self):
        """The linearized operator about the laminar flow (base U = sin(n y) + U0)."""
        return self.linearized_about(self.omega_lam)


# ---- selective frequency damping -------------------------------------------------------
def sfd_coupling(chi, delta, h):
    """Exact solution over h of X' = -chi (X - Y), Y' = (X - Y)/Delta as the 2 x 2
    matrix applied to (X, Y) pointwise."""
    B = np.array([[-chi, chi], [1.0 / delta, -1.0 / delta]])
    return sl.expm(h * B)


def sfd_step(step, E, X, Y):
    """One Strang-split step of the extended system: half the coupling (E =
    sfd_coupling(chi, Delta, h/2)), one step of the original system, half the
    coupling."""
    X, Y = E[0, 0] * X + E[0, 1] * Y, E[1, 0] * X + E[1, 1] * Y
    X = step(X)
    return E[0, 0] * X + E[0, 1] * Y, E[1, 0] * X + E[1, 1] * Y


def sfd(step, x0, chi, delta, h, check_every, tol, max_checks, norm=np.linalg.norm):
    """Selective frequency damping by encapsulated splitting.  ``step`` advances X
    by one time step h of the original system; the filtered state Y starts at
    X.  After every ``check_every`` controlled steps the residual of the
    original system, ||step(X) - X|| / h (that step is not applied), is
    recorded; the run stops when it is <= tol.  Returns (X, residual history,
    controlled steps taken)."""
    E = sfd_coupling(chi, delta, 0.5 * h)
    X = np.array(x0, dtype=float, copy=True)
    Y = X.copy()
    hist = []
    steps = 0
    for _ in range(max_checks):
        for _ in range(check_every):
            X, Y = sfd_step(step, E, X, Y)
            steps += 1
        Xn = step(X)
        res = norm(Xn - X) / h
        hist.append(res)
        if res <= tol:
            break
    return X, np.array(hist), steps


# ---- recursive projection method --------------------------------------------------------
def rpm(G, x0, U, H, tol, max_iter, norm=np.linalg.norm):
    """RPM iteration (Sec. 3.1.2) with a fixed basis U (n x p, orthonormal) and
    H = U^T M U.  Returns (x, residual history, iterations); the residual of
    iterate k is ||G(x~_k) - x~_k||."""
    x = np.array(x0, dtype=float, copy=True)
    p = U.shape[1]
    A = np.eye(p) - H
    hist = []
    for k in range(max_iter):
        xn = G(x)
        r = xn - x
        hist.append(norm(r))
        if hist[-1] <= tol:
            return x, np.array(hist), k
        z = U.T @ r
        c = np.linalg.solve(A, z)
        x = xn - U @ z + U @ c
    return x, np.array(hist), max_iter


def unstable_basis(apply_M, v0, m, k, delta):
    """U and H = U^T M U for RPM: an m-step Arnoldi factorisation of the Jacobian
    M, then the ordered real Schur form of H_m with the Ritz values |mu| >= 1 -
    delta (at least k of them) leading (the Krylov-Schur contraction of
    ``oracle.krylov_schur``).  Returns (U, H_p, kept Ritz values)."""
    from oracle.arnoldi import arnoldi
    from oracle.krylov_schur import kept_count
    a = arnoldi(apply_M, v0, m, m, 0.0)
    Hm = a["H"][:m, :m].real
    mu = np.linalg.eigvals(Hm)
    p, keep = kept_count(mu, k, m, delta, m - 2)
    wanted = lambda re, im: int(np.argmin(np.abs(mu - (re + 1j * im)))) in set(keep)
    S, Q, sdim = sl.schur(Hm, output="real", sort=wanted)
    U = a["V"][:m].real.T @ Q[:, :p]
    return U, S[:p, :p], mu[keep]


# ---- BoostConv --------------------------------------------------------------------------
def boostconv(G, x0, m, tol, max_iter, norm=np.linalg.norm, conds=None):
    """BoostConv iteration (Sec. 3.1.3): x~_{k+1} = x~_k + xi_k with
    xi_k = r_k - Y c + X c, c = Y^+ r_k (the least-squares solution, from the
    pseudo-inverse), from the last m pairs (X: applied corrections xi_j, Y:
    residual decrements r_j - r_{j+1}).  If ``conds`` is a list, the 2-norm
    condition number of Y at each correction is appended to it."""
    x = np.array(x0, dtype=float, copy=True)
    Xs, Ys = [], []
    hist = []
    r_prev = xi_prev = None
    for k in range(max_iter):
        r = G(x) - x
        hist.append(norm(r))
        if hist[-1] <= tol:
            return x, np.array(hist), k
        if r_prev is not None:
            Xs.append(xi_prev)
            Ys.append(r_prev - r)
            if len(Xs) > m:
                Xs.pop(0)
                Ys.pop(0)
        if Xs:
            X = np.stack(Xs, axis=1)
            Y = np.stack(Ys, axis=1)
            c = np.linalg.lstsq(Y, r, rcond=None)[0]
            if conds is not None:
                conds.append(float(np.linalg.cond(Y)))
            xi = r - Y @ c + X @ c
        else:
            xi = r
        x = x + xi
        r_prev, xi_prev = r, xi
    return x, np.array(hist), max_iter
