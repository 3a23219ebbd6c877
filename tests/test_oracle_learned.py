"""Pins of the learned-start data oracle (oracle/learned.py)."""
import numpy as np
import pytest

from oracle import learned as L
from oracle.kolmogorov import Kolmogorov
import workloads as W


@pytest.mark.parametrize("N", [16, 48, 96])
def test_packing_parseval_and_roundtrip(N):
    op = Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.005, 1.0)
    w = op.project(W.normal_real((N, N), N))
    v = L.pack(op.to_spectral(w), N)
    M = L.cutoff(N)
    assert v.size == 4 * M * (M + 1)
    # Parseval: the packed norm is the RMS of the (projected) field
    assert abs(np.linalg.norm(v) - np.sqrt(np.mean(w ** 2))) <= 1e-13 * np.linalg.norm(v)
    # round trip through rfft2 coordinates
    back = op.to_physical(L.unpack(v, N))
    assert np.max(np.abs(back - w)) <= 1e-13 * np.max(np.abs(w))


def _mode_vector(N, jx, seed, spread=6):
    """A packed real vector supported on one column (an x-translation family)."""
    M = L.cutoff(N)
    modes = L.packed_modes(N)
    rng = np.random.default_rng(seed)
    v = np.zeros(2 * len(modes))
    for i, (x, y) in enumerate(modes):
        if x == jx and abs(y) <= spread:
            v[2 * i], v[2 * i + 1] = rng.standard_normal(2) * np.exp(-abs(y) / 3)
    return v


def _shift(v, N, theta):
    """x-translation: coefficient (jx, jy) times exp(i jx theta)."""
    c = v[0::2] + 1j * v[1::2]
    jx = np.array([x for x, _ in L.packed_modes(N)])
    c = c * np.exp(1j * jx * theta)
    out = np.empty_like(v)
    out[0::2], out[1::2] = c.real, c.imag
    return out


@pytest.mark.parametrize("jx", [0, 1, 5, 31])
def test_target_invariant_under_translation_scale_and_sign(jx):
    N = 128
    v = _mode_vector(N, jx, 10 + jx)
    t0 = L.ritz_block_target(v[None, :].astype(complex), N)
    assert abs(np.linalg.norm(t0) - 1.0) < 1e-12
    for theta, scale in ((0.7, 3.0 + 0.0j), (2.1, -0.5 + 0.0j), (-1.3, 2.0j), (0.0, -1.0 + 0.0j)):
        z = _shift(v, N, theta if jx > 0 else 0.0) * scale
        t = L.ritz_block_target(z[None, :], N)
        assert np.max(np.abs(t - t0)) <= 1e-12, (theta, scale)
    # the pivot is real positive in the canonical form (sign only for kx = 0)
    c = t0[0::2] + 1j * t0[1::2]
    piv = np.argmax(np.abs(c))
    assert c[piv].real > 0
    if jx > 0:
        assert abs(c[piv].imag) <= 1e-14 * abs(c[piv])


def test_target_sums_modes_and_respects_use_mask():
    N = 96
    a, b = _mode_vector(N, 3, 1), _mode_vector(N, 7, 2)
    Z = np.stack([a, b]).astype(complex)
    ta = L.ritz_block_target(Z[:1], N)
    tb = L.ritz_block_target(Z[1:], N)
    both = L.ritz_block_target(Z, N)
    assert np.allclose(both, (ta + tb) / np.linalg.norm(ta + tb), atol=1e-14)
    assert np.allclose(L.ritz_block_target(Z, N, use=[0, 1]), tb, atol=1e-14)
    assert not np.any(L.ritz_block_target(Z, N, use=[0, 0]))


def test_decode_roundtrip_and_fallback():
    N = 128
    v = _mode_vector(N, 4, 3)
    t = L.ritz_block_target(v[None, :].astype(complex), N)
    r = W.normal_real(v.size, 4)
    v0, used = L.decode_start(t, r, N, 0.0)
    assert used == 1 and abs(np.linalg.norm(v0) - 1) < 1e-12
    # the decoded vector is a translated, scaled copy of the mode: its target is t again
    assert np.max(np.abs(L.ritz_block_target(v0[None, :].astype(complex), N) - t)) <= 1e-12
    # positions outside the state (jx = 0, jy <= 0) are ignored
    y = np.zeros(L.BLOCK)
    y[2 * L.block_slot(0, -3)] = 1.0
    v1, used = L.decode_start(y, r, N, 0.3)
    assert used == 0 and np.allclose(v1, r / np.linalg.norm(r))
    y[0] = np.nan
    assert L.decode_start(y, r, N, 0.3)[1] == 0
    # mixing weight
    v2, used = L.decode_start(t, r, N, 0.5)
    assert used == 1 and abs(np.dot(v2 - v0, r) / np.linalg.norm(r) - 0.5) < 1e-12
