"""Pins of the start-vector network oracle (oracle/mlp.py)."""
import numpy as np

from oracle import mlp
import workloads as W


def test_bf16_rounding_bit_patterns():
    # 1 + 2^-8 is halfway between two bfloat16 values (1 and 1 + 2^-7): ties to even -> 1
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above the halfway point rounds up
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    # exactly representable values are unchanged, sign is kept
    for v in (0.0, -2.0, 0.5, 3.0, -0.15625):
        assert mlp.bf16(v) == v
    # 8 significant bits: unit roundoff 2^-8 (plus the FP32 rounding on the way)
    x = W.normal_real(10000, 1) * 10.0 ** W.normal_real(10000, 2)
    err = np.abs(mlp.bf16(x) - x) / np.abs(x)
    assert np.all(err <= 2.0 ** -8 + 2.0 ** -24)
    assert err.max() > 2.0 ** -9          # the bound is attained, not slack by 2x


def test_backward_matches_central_differences_unquantised():
    P = mlp.init_params(3, width=16, out=24)
    X = W.normal_real((5, 2), 4)
    T = W.normal_real((5, 24), 5)
    G, _ = mlp.grads(P, X, T, quantize=False)
    rng = np.random.default_rng(6)
    h = 1e-6
    for key in mlp.ORDER:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in P[key].shape)
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[key][idx] += h
            Pm[key][idx] -= h
            fd = (mlp.loss(Pp, X, T, False) - mlp.loss(Pm, X, T, False)) / (2 * h)
            assert abs(fd - G[key][idx]) <= 1e-7 * max(1.0, abs(fd)), (key, idx, fd, G[key][idx])


def test_quantised_gradients_close_to_exact():
    P = mlp.init_params(7)
    X = W.normal_real((8, 2), 8)
    T = 0.1 * W.normal_real((8, mlp.OUT), 9)
    Gq, _ = mlp.grads(P, X, T, True)
    Ge, _ = mlp.grads(P, X, T, False)
    for k in mlp.ORDER:
        rel = np.linalg.norm(Gq[k] - Ge[k]) / np.linalg.norm(Ge[k])
        assert rel < 2e-2, (k, rel)


def test_adam_decreases_loss_and_flatten_roundtrip():
    P = mlp.init_params(11, width=32, out=40)
    X = W.normal_real((16, 2), 12)
    T = np.tanh(X @ W.normal_real((2, 40), 13))
    st = {}
    l0 = mlp.loss(P, X, T)
    for t in range(1, 201):
        G, _ = mlp.grads(P, X, T)
        P = mlp.adam_step(P, G, st, t, 1e-2)
    assert mlp.loss(P, X, T) < 0.2 * l0
    v = mlp.flatten(P)
    Q = mlp.unflatten(v, width=32, out=40)
    assert all(np.array_equal(P[k], Q[k]) for k in mlp.ORDER)
