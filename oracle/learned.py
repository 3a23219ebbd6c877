"""Oracle: the low-mode block that the start-vector network predicts -- packed
spectral coordinates, the training target made from Ritz vectors, and the
start vector assembled from a prediction.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Algorithm 1 (Sec. 3.2.1) accepts any start vector; a start vector with large
components along the wanted eigenvectors shortens the Krylov sequence.  This
module is the data side of a learned start, which is not part of the paper.

Packed spectral state of the Navier-Stokes operator (the library's state
vector): n = 4 M (M + 1) reals, M = (N - 1) // 3; first the kx = 0 column with
jy = 1..M, then the columns jx = 1..M with jy = -M..M; each complex coefficient
is sqrt(2) rfft2(omega)[jy mod N, jx] / N^2 stored as (re, im).  Its Euclidean
norm equals the RMS of the physical field (Parseval).

Low-mode block: the 32 x 32 coefficients jx in [0, 32), jy in [-16, 16), as
2048 reals, output index 2 (32 jx + jy + 16) + c (c = 0 re, 1 im).  Positions
that the state does not hold (jx = 0 with jy <= 0, or |jx|, |jy| > M) are
unused.

Target of one instance, from its wanted Ritz vectors z_s (complex n-vectors over
the packed reals), in the wanted order, those flagged in ``use`` only:
  a = Re z (Im z when ||Im z|| > ||Re z||): a real vector of the eigenspace;
  c = complex coefficients of a; restricted to the block (skipped when zero);
  pivot = smallest packed index among the block coefficients with
          |c|^2 >= (1 - 1e-6) max |c|^2;
  canonical form: an x-translation makes the pivot real positive (coefficient
  (jx, jy) times exp(-i jx phi / jx_p), phi = arg c_pivot) when jx_p > 0, a
  sign flip making Re c_pivot >= 0 when jx_p = 0;
  the canonical block is scaled to unit norm and added to the sum.
The target is the sum scaled to unit norm (zero if nothing was added).

Start vector from a prediction y (2048 reals) and a random state r:
  p = y scattered to the packed positions it covers (zero elsewhere);
  v0 = p / ||p|| + gamma r / ||r||, or r / ||r|| when ||p|| is zero or not
  finite (the random-start fallback).

Parity status: pinned -- Parseval and the rfft2 round trip for the packing,
invariance of the target under x-translation, complex scaling and sign of the
input mode, and the block/packing round trip; see tests/test_oracle_learned.py.
"""
from __future__ import annotations

import numpy as np

BJX = 32
BJY0, BJY1 = -16, 16
BLOCK = 2 * BJX * (BJY1 - BJY0)
TIE = 1e-6


def cutoff(N):
    return (N - 1) // 3


def packed_modes(N):
    """(jx, jy) of each complex coefficient of the packed state, in state order."""
    M = cutoff(N)
    return [(0, jy) for jy in range(1, M + 1)] + [(jx, jy) for jx in range(1, M + 1) for jy in range(-M, M + 1)]


def pack(wh, N):
    """rfft2 array (N x N//2+1) -> packed real state."""
    c = np.array([wh[jy % N, jx] for jx, jy in packed_modes(N)]) * np.sqrt(2.0) / N ** 2
    out = np.empty(2 * len(c))
    out[0::2], out[1::2] = c.real, c.imag
    return out


def unpack(v, N):
    """Packed real state -> rfft2 array with the conjugate symmetry of the kx = 0
    column filled in."""
    wh = np.zeros((N, N // 2 + 1), dtype=complex)
    c = (v[0::2] + 1j * v[1::2]) * N ** 2 / np.sqrt(2.0)
    for (jx, jy), val in zip(packed_modes(N), c):
        wh[jy % N, jx] = val
        if jx == 0:
            wh[(-jy) % N, 0] = np.conj(val)
    return wh


def block_slot(jx, jy):
    """Complex slot (0..1023) of mode (jx, jy) in the block, or -1."""
    if 0 <= jx < BJX and BJY0 <= jy < BJY1:
        return BJX * 0 + jx * (BJY1 - BJY0) + (jy - BJY0)
    return -1


def ritz_block_target(Z, N, use=None):
    """Training target (2048 reals) from the rows of Z (k x n complex)."""
    modes = packed_modes(N)
    slots = np.array([block_slot(jx, jy) for jx, jy in modes])
    jxs = np.array([jx for jx, _ in modes])
    inb = np.nonzero(slots >= 0)[0]
    acc = np.zeros(BLOCK // 2, dtype=complex)
    for s, z in enumerate(np.atleast_2d(Z)):
        if use is not None and not use[s]:
            continue
        a = z.imag if np.sum(z.imag ** 2) > np.sum(z.real ** 2) else z.real
        c = a[0::2] + 1j * a[1::2]
        cb = c[inb]
        mag = np.abs(cb) ** 2
        if not np.any(mag > 0):
            continue
        piv = inb[np.nonzero(mag >= (1.0 - TIE) * mag.max())[0][0]]
        jp, cp = jxs[piv], c[piv]
        if jp > 0:
            rot = np.exp(-1j * jxs[inb] * np.angle(cp) / jp)
        else:
            rot = np.full(len(inb), 1.0 if cp.real >= 0 else -1.0)
        b = rot * cb
        acc[slots[inb]] += b / np.linalg.norm(b)
    nrm = np.linalg.norm(acc)
    if nrm > 0:
        acc /= nrm
    out = np.empty(BLOCK)
    out[0::2], out[1::2] = acc.real, acc.imag
    return out


def decode_start(y, r, N, gamma):
    """Start vector from a prediction y and a random state r; returns (v0, used)."""
    modes = packed_modes(N)
    p = np.zeros(2 * len(modes))
    for i, (jx, jy) in enumerate(modes):
        sl = block_slot(jx, jy)
        if sl >= 0:
            p[2 * i] = y[2 * sl]
            p[2 * i + 1] = y[2 * sl + 1]
    pn = np.linalg.norm(p)
    rn = np.linalg.norm(r)
    if not np.isfinite(pn) or pn == 0.0:
        return r / rn, 0
    return p / pn + gamma * r / rn, 1
