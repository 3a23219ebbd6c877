"""Start-vector network on the GPU (bfloat16 MFMA forward/backward, Adam)
against the FP64 oracle with the same bfloat16 rounding points."""
import numpy as np
import pytest
import torch

from oracle import mlp
import workloads as W

pytestmark = pytest.mark.gpu

# Tolerances.  Both sides round the same operands to bfloat16; they differ by
# FP32 (GPU) versus FP64 (oracle) arithmetic before the rounding, which moves
# an operand to the neighbouring bfloat16 value only when it lies within about
# 1e-7 relative of a rounding midpoint, and by FP32 accumulation order.
FWD_TOL = 2e-4      # max |dY| / max |Y|
GRAD_TOL = 2e-3     # ||dg|| / ||g|| per parameter block
STEP_TOL = 2e-2     # ||w_gpu - w_oracle|| / ||w_oracle - w_0|| after Adam steps


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    raw = np.stack([rng.uniform(5.0, 40.0, B), rng.choice(W.BATCH_ALPHAS, B)], 1).astype(np.float32)
    return raw


def _net(tsk, width, seed):
    P = mlp.init_params(seed, width)
    net = tsk.mlp_create(width)
    tsk.mlp_set_params(net, mlp.flatten(P).astype(np.float32))
    return net, P


def test_device_init_matches_oracle_bitwise(tsk):
    for width in (48, 512):
        net = tsk.mlp_create(width)
        tsk.mlp_init(net, 1234)
        got = tsk.mlp_get_params(net)
        want = mlp.flatten(mlp.init_params(1234, width)).astype(np.float32)
        assert got.shape == want.shape
        assert np.array_equal(got, want), width


@pytest.mark.parametrize("width,B", [(512, 64), (512, 37), (512, 1), (48, 5), (96, 130)])
def test_forward_matches_oracle(tsk, width, B):
    net, P = _net(tsk, width, 7)
    raw = _inputs(B, 8)
    Y = tsk.mlp_forward(net, torch.from_numpy(raw).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = mlp.forward(P, mlp.features(raw.astype(np.float64)))
    err = np.max(np.abs(Y - ref)) / np.max(np.abs(ref))
    assert err <= FWD_TOL, err


@pytest.mark.parametrize("width,B", [(512, 64), (512, 37), (48, 5)])
def test_gradients_match_oracle(tsk, width, B):
    net, P = _net(tsk, width, 11)
    raw = _inputs(B, 12)
    T = (0.1 * W.normal_real((B, mlp.OUT), 13)).astype(np.float32)
    g, loss = tsk.mlp_gradients(net, torch.from_numpy(raw).cuda(), torch.from_numpy(T).cuda())
    G = mlp.unflatten(g.cpu().numpy().astype(np.float64), width)
    Gr, loss_r = mlp.grads(P, mlp.features(raw.astype(np.float64)), T.astype(np.float64))
    assert abs(loss - loss_r) <= 1e-5 * loss_r
    for k in mlp.ORDER:
        rel = np.linalg.norm(G[k] - Gr[k]) / np.linalg.norm(Gr[k])
        assert rel <= GRAD_TOL, (k, rel)


def test_adam_steps_match_oracle_and_are_reproducible(tsk):
    width, B, steps, lr = 512, 64, 3, 1e-3
    raw = _inputs(B, 21)
    T = (0.1 * W.normal_real((B, mlp.OUT), 22)).astype(np.float32)
    x, t = torch.from_numpy(raw).cuda(), torch.from_numpy(T).cuda()
    net, P = _net(tsk, width, 20)
    w0 = mlp.flatten(P)
    losses = tsk.mlp_train(net, x, t, steps, lr)
    w_gpu = tsk.mlp_get_params(net).astype(np.float64)
    X = mlp.features(raw.astype(np.float64))
    st, Pr, lr_ = {}, {k: v.copy() for k, v in P.items()}, []
    for i in range(1, steps + 1):
        G, l = mlp.grads(Pr, X, T.astype(np.float64))
        lr_.append(l)
        Pr = mlp.adam_step(Pr, G, st, i, lr)
    w_or = mlp.flatten(Pr)
    assert np.allclose(losses, lr_, rtol=1e-5, atol=0)
    rel = np.linalg.norm(w_gpu - w_or) / np.linalg.norm(w_or - w0)
    assert rel <= STEP_TOL, rel
    # same parameters and data give the same bits
    net2, _ = _net(tsk, width, 20)
    losses2 = tsk.mlp_train(net2, x, t, steps, lr)
    assert np.array_equal(losses, losses2)
    assert np.array_equal(tsk.mlp_get_params(net2), tsk.mlp_get_params(net))


def test_training_reduces_loss(tsk):
    width, B = 512, 64
    raw = _inputs(B, 31)
    X = mlp.features(raw.astype(np.float64))
    # a smooth target of the inputs
    T = np.tanh(X @ W.normal_real((2, mlp.OUT), 32)).astype(np.float32) * 0.1
    net = tsk.mlp_create(width)
    tsk.mlp_init(net, 5)
    losses = tsk.mlp_train(net, torch.from_numpy(raw).cuda(), torch.from_numpy(T).cuda(), 300, 1e-3)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.05 * losses[0], (losses[0], losses[-1])


def test_rejects_bad_arguments(tsk):
    net = tsk.mlp_create(64)
    x = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(tsk.TskError) as e:   # parameters not set yet
        tsk.mlp_forward(net, x)
    assert e.value.status == tsk.TSK_ESTATE
    tsk.mlp_init(net, 0)
    t = torch.zeros((4, mlp.OUT), dtype=torch.float32, device="cuda")
    with pytest.raises(tsk.TskError) as e:
        tsk.mlp_train(net, x, t, 1, -1.0)
    assert e.value.status == tsk.TSK_EINVAL
    big = torch.zeros((4097, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(tsk.TskError):
        tsk.mlp_forward(net, big)
