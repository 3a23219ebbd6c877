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


def test_adam_first_step_closed_form():
    # Kingma & Ba (2015), Algorithm 1: after one step the bias-corrected moments
    # are exactly g and g^2, so the update is -lr g / (|g| + eps) elementwise:
    # about lr in size whatever the scale of g, and lr/2 at |g| = eps.  A missing
    # bias correction would shrink it by (1 - b1) / sqrt(1 - b2) ~ 3.2; eps inside
    # the square root would give lr g / sqrt(g^2 + eps) = lr 1e-4 at |g| = eps.
    g = np.array([3.0, -2e-3, 1e-8, -1e-8, 5e4, 0.0])
    P = {"w": np.zeros_like(g)}
    mlp.adam_step(P, {"w": g}, {}, 1, 0.01)
    want = np.array([-0.01, 0.01, -0.005, 0.005, -0.01, 0.0])
    want[0] *= 3.0 / (3.0 + 1e-8)
    want[1] *= 2e-3 / (2e-3 + 1e-8)
    want[4] *= 5e4 / (5e4 + 1e-8)
    assert np.allclose(P["w"], want, rtol=1e-12, atol=0.0)


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient both bias-corrected moments stay exactly g and g^2
    # at every t, so each step moves each parameter by lr g / (|g| + eps)
    g = np.array([0.7, -4.0, 2.5e-6])
    P = {"w": np.ones(3)}
    st = {}
    for t in range(1, 51):
        P = mlp.adam_step(P, {"w": g}, st, t, 1e-3)
    want = 1.0 - 50 * 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(P["w"], want, rtol=0.0, atol=1e-13)


def test_adam_two_steps_by_hand():
    # b1 = 1/2, b2 = 3/4, eps = 0, lr = 1, w0 = 0, gradients 2 then 4.
    # t = 1: m = 1, v = 1, m^ = 1/(1/2) = 2, v^ = 1/(1/4) = 4, w = -2/2 = -1.
    # t = 2: m = 1/2 + 2 = 5/2, v = 3/4 + 4 = 19/4, m^ = (5/2)/(3/4) = 10/3,
    #        v^ = (19/4)/(7/16) = 76/7, w = -1 - (10/3) sqrt(7/76).
    P = {"w": np.zeros(1)}
    st = {}
    P = mlp.adam_step(P, {"w": np.array([2.0])}, st, 1, 1.0, b1=0.5, b2=0.75, eps=0.0)
    assert P["w"][0] == -1.0
    P = mlp.adam_step(P, {"w": np.array([4.0])}, st, 2, 1.0, b1=0.5, b2=0.75, eps=0.0)
    assert abs(P["w"][0] - (-1.0 - (10.0 / 3.0) * np.sqrt(7.0 / 76.0))) <= 1e-15
