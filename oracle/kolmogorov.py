"""Oracle: linearized 2D incompressible Navier-Stokes about a base flow, vorticity form,
pseudo-spectral in a doubly periodic box, integrating-factor RK4 time stepper.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Paper: Sec. 3, eq. "linearized Navier-Stokes equations": the perturbation u about
a base flow U_b obeys du/dt + (u.grad)U_b + (U_b.grad)u = -grad p + Re^-1 lap u,
div u = 0.  Taking the curl in 2D with the perturbation streamfunction psi
(u = d psi/dy, v = -d psi/dx, -lap psi = omega) gives

    d omega/dt = -(U d_x omega + V d_y omega + u d_x Omega + v d_y Omega) + Re^-1 lap omega,

with Omega = d_x V - d_y U the base vorticity.  The paper uses a time-stepper of
this equation as the black-box matvec of the exponential propagator
M = exp(A T) (Sec. 3, "time-stepper approach"; Sec. 3.2).

Discretisation (the workload's reading): box x in [0, 2 pi/alpha), y in [0, 2 pi),
N x N grid, arrays indexed [y, x]; rfft2 over (y, x) so kx = alpha*jx on the
last axis.  Products are formed in physical space.  2/3 rule: keep |jx| < N/3 and
|jy| < N/3 strictly, drop the mean (0, 0) mode.  Time: Lawson's integrating
factor RK4 with E(h) = exp(-K^2 h / Re).  The base flow is any (U, V) with the
gradient of its vorticity (Omega_x, Omega_y) on the grid; the Kolmogorov base
U = (sin(n y), 0) gives Omega = -n cos(n y), Omega_x = 0, Omega_y = n^2 sin(n y).

State representation: the real physical vorticity field (N*N reals) with the
plain Euclidean inner product over grid points (Sec. 2.3.1 uses the Euclidean
inner product).

Parity status: pinned -- pseudo-spectral right-hand side against a brute-force
spectral convolution (general base flow, tiny grid) and against the closed-form
Galerkin coupling of the sinusoidal base; a reflection symmetry ties the V and
Omega_x terms to the U and Omega_y terms; eigenvalues against dense eig of the
assembled Galerkin blocks; see tests/test_oracle_kolmogorov.py.
"""
from __future__ import annotations

import numpy as np


def dealias_cutoff(N):
    """Largest kept |j| under the strict 2/3 rule |j| < N/3."""
    return (N - 1) // 3


class Kolmogorov:
    def __init__(self, N, alpha, Re, dt, T, U, V, Ox, Oy):
        self.N = int(N)
        self.alpha = float(alpha)
        self.Re = float(Re)
        self.dt = float(dt)
        self.T = float(T)
        nsteps = self.T / self.dt
        self.nsteps = int(round(nsteps))
        if abs(nsteps - self.nsteps) > 1e-9 * max(1.0, nsteps):
            raise ValueError("T must be an integer multiple of dt")
        N = self.N
        self.U = np.asarray(U, dtype=float).reshape(N, N)
        self.V = np.asarray(V, dtype=float).reshape(N, N)
        self.Ox = np.asarray(Ox, dtype=float).reshape(N, N)
        self.Oy = np.asarray(Oy, dtype=float).reshape(N, N)
        jx = np.arange(N // 2 + 1)
        jy = np.fft.fftfreq(N, 1.0 / N)
        self.kx = (self.alpha * jx)[None, :]
        self.ky = jy[:, None].astype(float)
        self.K2 = self.kx ** 2 + self.ky ** 2
        M = dealias_cutoff(N)
        self.mask = (np.abs(jx)[None, :] <= M) & (np.abs(jy)[:, None] <= M)
        self.mask[0, 0] = False
        with np.errstate(divide="ignore"):
            self.invK2 = np.where(self.K2 > 0, 1.0 / np.where(self.K2 > 0, self.K2, 1.0), 0.0)

    @classmethod
    def kolmogorov(cls, N, alpha, Re, dt, T, n_forcing=4):
        """Kolmogorov base flow U = (sin(n y), 0) (held steady by a body force,
        which cancels from the linear equation)."""
        y = 2 * np.pi * np.arange(N) / N
        Y = np.repeat(y[:, None], N, axis=1)
        n = float(n_forcing)
        U = np.sin(n * Y)
        V = np.zeros_like(U)
        Ox = np.zeros_like(U)
        Oy = n * n * np.sin(n * Y)
        return cls(N, alpha, Re, dt, T, U, V, Ox, Oy)

    # ---- grids -------------------------------------------------------------
    def grid(self):
        N = self.N
        x = 2 * np.pi * np.arange(N) / (self.alpha * N)
        y = 2 * np.pi * np.arange(N) / N
        return x, y

    # ---- spectral <-> physical --------------------------------------------
    def to_spectral(self, w):
        return np.fft.rfft2(np.asarray(w, dtype=float).reshape(self.N, self.N)) * self.mask

    def to_physical(self, wh):
        return np.fft.irfft2(wh, s=(self.N, self.N))

    def project(self, w):
        """Orthogonal projection of a physical field on the dealiased, zero-mean
        subspace the time-stepper lives in."""
        return self.to_physical(self.to_spectral(w))

    # ---- right-hand side ----------------------------------------------------
    def advection_hat(self, wh):
        """Dealiased Fourier transform of the linearized advection
        -(U w_x + V w_y + u Omega_x + v Omega_y) (Sec. 3, linearized N-S in
        vorticity form), products taken on the grid."""
        psih = wh * self.invK2
        irf = lambda f: np.fft.irfft2(f, s=(self.N, self.N))
        wx = irf(1j * self.kx * wh)
        wy = irf(1j * self.ky * wh)
        u = irf(1j * self.ky * psih)
        v = irf(-1j * self.kx * psih)
        P = self.U * wx + self.V * wy + u * self.Ox + v * self.Oy
        return -np.fft.rfft2(P) * self.mask

    def rhs_hat(self, wh):
        """Full linear right-hand side A w in spectral form (advection + viscous)."""
        return self.advection_hat(wh) - (self.K2 / self.Re) * wh * self.mask

    # ---- integrating-factor RK4 (Lawson) -------------------------------------
    def step_hat(self, wh):
        """One Lawson integrating-factor RK4 step of size h = dt: the viscous
        term is integrated exactly by E(t) = exp(-K^2 t / Re), classical RK4 is
        applied to the advection term in the variable E(-t) w."""
        h = self.dt
        E1 = np.exp(-self.K2 * h / self.Re)
        Eh = np.exp(-self.K2 * (h / 2) / self.Re)
        Nf = self.advection_hat
        a = Nf(wh)
        b = Nf(Eh * (wh + (h / 2) * a))
        c = Nf(Eh * wh + (h / 2) * b)
        d = Nf(E1 * wh + h * Eh * c)
        return E1 * wh + (h / 6) * (E1 * a + 2 * Eh * (b + c) + d)

    def apply(self, w):
        """Matvec of the exponential propagator (Sec. 3.2): march the linearized
        equation over T = nsteps * dt.  Physical field in, physical field out."""
        wh = self.to_spectral(w)
        for _ in range(self.nsteps):
            wh = self.step_hat(wh)
        return self.to_physical(wh)

    # ---- helpers for pins ----------------------------------------------------
    def kept_modes(self):
        """List of (iy, jx) indices of the rfft2 array that the state keeps."""
        return np.argwhere(self.mask)


def base_vorticity_gradient(U, V, alpha):
    """Gradient (Omega_x, Omega_y) of the base vorticity Omega = V_x - U_y, by
    spectral differentiation of grid fields (all resolved modes, Nyquist zeroed)."""
    U = np.asarray(U, float)
    V = np.asarray(V, float)
    N = U.shape[0]
    jx = np.arange(N // 2 + 1).astype(float)
    jy = np.fft.fftfreq(N, 1.0 / N)
    if N % 2 == 0:
        jx[-1] = 0.0
        jy = jy.copy()
        jy[N // 2] = 0.0
    kx = alpha * jx[None, :]
    ky = jy[:, None]
    Uh = np.fft.rfft2(U)
    Vh = np.fft.rfft2(V)
    Oh = 1j * kx * Vh - 1j * ky * Uh
    irf = lambda f: np.fft.irfft2(f, s=(N, N))
    return irf(1j * kx * Oh), irf(1j * ky * Oh)


def galerkin_sinusoidal_advection(op: Kolmogorov, wh, n_forcing=4):
    """Closed-form Fourier coupling of the advection term for U = (sin(n y), 0):
    the term reduces to -sin(n y) d_x(omega - n^2 psi), whose transform at
    (kx, ky) is -(kx/2) [g(ky-n) - g(ky+n)] with g = w_hat (1 - n^2/K^2).
    Independent of the grid products in ``advection_hat``; used as a pin."""
    N = op.N
    n = int(n_forcing)
    g = wh * op.mask * (1.0 - n * n * op.invK2)
    g = np.where(op.mask, g, 0)
    out = np.zeros_like(wh)
    jy = np.fft.fftfreq(N, 1.0 / N).astype(int)
    index = {int(j): i for i, j in enumerate(jy)}
    for i, j in enumerate(jy):
        lo = index.get(int(j) - n)
        hi = index.get(int(j) + n)
        acc = np.zeros(wh.shape[1], dtype=complex)
        if lo is not None and abs(int(j) - n) < N // 2:
            acc += g[lo]
        if hi is not None and abs(int(j) + n) < N // 2:
            acc -= g[hi]
        out[i] = -(op.kx[0] / 2.0) * acc
    return out * op.mask


def galerkin_sinusoidal_blocks(N, alpha, Re, n_forcing=4):
    """Dense Galerkin matrices of A restricted to each kx column (the operator is
    block diagonal in kx for a base flow that depends on y only).  Returns a dict
    jx -> (jy list, matrix) over the kept modes."""
    M = dealias_cutoff(N)
    n = int(n_forcing)
    blocks = {}
    for jx in range(0, M + 1):
        kx = alpha * jx
        jys = [j for j in range(-M, M + 1) if not (jx == 0 and j == 0)]
        pos = {j: i for i, j in enumerate(jys)}
        A = np.zeros((len(jys), len(jys)))
        for j in jys:
            K2 = kx * kx + j * j
            A[pos[j], pos[j]] = -K2 / Re
            for src, sgn in ((j - n, -1.0), (j + n, +1.0)):
                if src in pos:
                    K2s = kx * kx + src * src
                    A[pos[j], pos[src]] += sgn * (kx / 2.0) * (1.0 - n * n / K2s)
        blocks[jx] = (jys, A)
    return blocks


def brute_force_advection(op: Kolmogorov, wh, base_modes):
    """Linearized advection by explicit convolution sums over Fourier modes of a
    band-limited base flow.  ``base_modes`` maps (jx, jy) -> complex coefficient
    of the base streamfunction Psi (physical Psi = sum c e^{i(kx x + ky y)}, real
    by including conjugates).  U = Psi_y, V = -Psi_x, Omega = -lap Psi.
    Direct O(modes^2) double loop; pins ``advection_hat`` for general bases."""
    N = op.N
    alpha = op.alpha
    M = dealias_cutoff(N)
    # Full (two-sided) perturbation coefficients c(jx, jy) from the rfft2 array,
    # normalised so that w = sum c e^{i k.x}.
    full = {}
    jyv = np.fft.fftfreq(N, 1.0 / N).astype(int)
    for iy, jy in enumerate(jyv):
        for jx in range(0, N // 2 + 1):
            if not op.mask[iy, jx]:
                continue
            c = wh[iy, jx] / (N * N)
            full[(jx, int(jy))] = c
            if jx > 0:
                full[(-jx, -int(jy))] = np.conj(c)
    out = {}
    for (bx, by), C in base_modes.items():
        kbx, kby = alpha * bx, float(by)
        Ub = 1j * kby * C          # U = Psi_y
        Vb = -1j * kbx * C         # V = -Psi_x
        Ob = (kbx ** 2 + kby ** 2) * C   # Omega = -lap Psi
        Obx = 1j * kbx * Ob
        Oby = 1j * kby * Ob
        for (px, py), c in full.items():
            kpx, kpy = alpha * px, float(py)
            K2 = kpx ** 2 + kpy ** 2
            wx = 1j * kpx * c
            wy = 1j * kpy * c
            psi = c / K2
            u = 1j * kpy * psi
            v = -1j * kpx * psi
            val = Ub * wx + Vb * wy + u * Obx + v * Oby
            key = (bx + px, by + py)
            out[key] = out.get(key, 0) - val
    res = np.zeros_like(wh)
    for iy, jy in enumerate(jyv):
        for jx in range(0, N // 2 + 1):
            if op.mask[iy, jx]:
                res[iy, jx] = out.get((jx, int(jy)), 0) * (N * N)
    return res


def base_from_streamfunction(base_modes, N, alpha):
    """Grid fields (U, V, Omega_x, Omega_y) of a band-limited base streamfunction
    given as in ``brute_force_advection`` (real part of the mode sum; modes must
    come with their conjugates)."""
    x = 2 * np.pi * np.arange(N) / (alpha * N)
    y = 2 * np.pi * np.arange(N) / N
    X, Y = np.meshgrid(x, y)
    U = np.zeros((N, N), complex)
    V = np.zeros((N, N), complex)
    Ox = np.zeros((N, N), complex)
    Oy = np.zeros((N, N), complex)
    for (bx, by), C in base_modes.items():
        kbx, kby = alpha * bx, float(by)
        e = C * np.exp(1j * (kbx * X + kby * Y))
        U += 1j * kby * e
        V += -1j * kbx * e
        Ob = (kbx ** 2 + kby ** 2)
        Ox += 1j * kbx * Ob * e
        Oy += 1j * kby * Ob * e
    return U.real, V.real, Ox.real, Oy.real
