"""Learned start vector on the GPU: the Ritz-vector training target and the
start-vector assembly against the oracle (seeded synthetic inputs)."""
import numpy as np
import pytest
import torch

from oracle import learned as L
from oracle import mlp
from oracle.kolmogorov import Kolmogorov
from oracle.rng import normal
import workloads as W

pytestmark = pytest.mark.gpu


def _kolmo(tsk, N, prec, Re=20.0, alpha=0.5):
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, 0.005, 1.0)
    tsk.set_base_kolmogorov(op, 4)
    return op


def _mode_rows(N, k, seed):
    """k synthetic 'Ritz vectors': single-column modes with random complex
    scale, one spread over all columns, and one with only an imaginary part."""
    modes = L.packed_modes(N)
    rng = np.random.default_rng(seed)
    n = 2 * len(modes)
    Z = np.zeros((k, n), dtype=complex)
    cols = rng.choice(np.arange(0, min(L.cutoff(N), 40)), size=k, replace=False)
    for s in range(k):
        v = np.zeros(n)
        for i, (jx, jy) in enumerate(modes):
            if jx == cols[s]:
                v[2 * i:2 * i + 2] = rng.standard_normal(2) * np.exp(-abs(jy) / 4.0)
        Z[s] = v * (rng.standard_normal() + 1j * rng.standard_normal())
    Z[-1] = 1j * rng.standard_normal(n)                 # imaginary part only, all columns
    if k > 2:
        Z[-2] = rng.standard_normal(n) + 0.3j * rng.standard_normal(n)
    return Z


@pytest.mark.parametrize("N,k", [(128, 6), (96, 3), (48, 4)])
def test_ritz_block_target_matches_oracle(tsk, N, k):
    op = _kolmo(tsk, N, tsk.TSK_FP32)
    Z = _mode_rows(N, k, N + k)
    use = [1] * k
    use[1] = 0
    for u in (None, use):
        got = tsk.ritz_block_target(op, torch.from_numpy(Z).cuda(), u).cpu().numpy().astype(np.float64)
        want = L.ritz_block_target(Z, N, u)
        assert np.max(np.abs(got - want)) <= 2e-7, (u, np.max(np.abs(got - want)))
    none = tsk.ritz_block_target(op, torch.from_numpy(Z).cuda(), [0] * k).cpu().numpy()
    assert not np.any(none)


@pytest.mark.parametrize("N,prec", [(128, 0), (128, 1), (48, 0)])
def test_start_vector_matches_oracle(tsk, N, prec):
    width, seed, Re, alpha, gamma = 512, 17, 23.5, 0.75, 0.3
    P = mlp.init_params(3, width)
    net = tsk.mlp_create(width)
    tsk.mlp_set_params(net, mlp.flatten(P).astype(np.float32))
    op = _kolmo(tsk, N, prec, Re, alpha)
    v0, used = tsk.mlp_start(net, op, Re, alpha, gamma, seed)
    assert used
    raw = np.array([[Re, alpha]], dtype=np.float32).astype(np.float64)
    y, _ = mlp.forward(P, mlp.features(raw))
    ref_op = Kolmogorov.kolmogorov(N, alpha, Re, 0.005, 1.0)
    phys = normal(N * N, seed).reshape(N, N)
    if prec == 1:
        phys = phys.astype(np.float32).astype(np.float64)
    r = L.pack(ref_op.to_spectral(phys), N)
    want, used_r = L.decode_start(y[0], r, N, gamma)
    assert used_r == 1
    got = v0.cpu().numpy().astype(np.float64)
    tol = 2e-4 if prec == 0 else 3e-4
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want)), np.max(np.abs(got - want))


def test_start_vector_falls_back_to_random(tsk):
    N, seed = 64, 5
    net = tsk.mlp_create(64)
    tsk.mlp_set_params(net, np.zeros(net.param_count, dtype=np.float32))   # predicts 0
    op = _kolmo(tsk, N, tsk.TSK_FP64)
    v0, used = tsk.mlp_start(net, op, 20.0, 0.5, 0.3, seed)
    assert not used
    ref_op = Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.005, 1.0)
    r = L.pack(ref_op.to_spectral(normal(N * N, seed).reshape(N, N)), N)
    assert np.allclose(v0.cpu().numpy(), r / np.linalg.norm(r), rtol=0, atol=1e-13)
    bad = np.zeros(net.param_count, dtype=np.float32)
    bad[net.param_count - mlp.OUT + 2 * (32 * 1 + 16)] = np.nan            # b3 at (jx, jy) = (1, 0)
    tsk.mlp_set_params(net, bad)
    v1, used = tsk.mlp_start(net, op, 20.0, 0.5, 0.3, seed)
    assert not used and torch.equal(v1, v0)
    cg = tsk.create_cgle1d()
    with pytest.raises(tsk.TskError):
        tsk.mlp_start(net, cg, 20.0, 0.5, 0.3, seed)


# ---- end to end: train on the sweep's Ritz vectors, judge on held-out (Re, alpha) ----
FP32_FLOOR = 32 * 2.0 ** -24        # FP32 residual floor of the stop rule (relative to |mu|)
FP32_LAMBDA_BOUND = 2e-5            # stated FP32 eigenvalue accuracy
GAMMA = 0.1


def _exact_top(c, k):
    """Leading k distinct eigenvalues of the linearized operator (dense eig of
    the Galerkin blocks), as (Re, |Im|) pairs: either member of a conjugate pair
    may be the one a run reports first."""
    from oracle.kolmogorov import galerkin_sinusoidal_blocks
    ev = []
    for jx, (jys, A) in galerkin_sinusoidal_blocks(c["N"], c["alpha"], c["Re"]).items():
        w = np.diag(A)[[i for i, j in enumerate(jys) if j > 0]] if jx == 0 else np.linalg.eigvals(A)
        ev.extend(w.tolist())
    ev = sorted(ev, key=lambda z: (-z.real, -z.imag))
    out = []
    for z in ev:
        if all(abs(z - y) > 1e-8 for y in out):
            out.append(z)
        if len(out) == k:
            break
    return np.array(out)


def _fold(lam):
    return np.array([complex(z.real, abs(z.imag)) for z in lam])


def _kop(tsk, c):
    op = tsk.create_kolmo2d(c["N"], tsk.TSK_FP32)
    tsk.set_params_kolmo(op, c["Re"], c["alpha"], c["dt"], c["T"])
    tsk.set_base_kolmogorov(op, c["n_forcing"])
    return op


def test_learned_start_saves_matvecs_on_heldout_instances(tsk):
    from conftest import match_sets
    sweep = W.learned_training_sweep()
    ops = [_kop(tsk, c) for c in sweep]
    res = tsk.batch_arnoldi(ops, sweep[0]["m"], sweep[0]["k"], sweep[0]["tol"], want_vectors=True)
    targets = []
    for c, op, r in zip(sweep, ops, res):
        use = [r["res"][i] <= max(c["tol"], FP32_FLOOR * abs(r["mu"][i])) for i in range(r["n_ritz"])]
        targets.append(tsk.ritz_block_target(op, r["X"], use))
    T = torch.stack(targets).contiguous()
    assert int((T.norm(dim=1) > 0.5).sum()) >= 60          # nearly every instance gave a target
    x = torch.tensor([[c["Re"], c["alpha"]] for c in sweep], dtype=torch.float32, device="cuda")
    net = tsk.mlp_create(512, W.LEARNED_IN_LO, W.LEARNED_IN_HI)
    tsk.mlp_init(net, 0)
    losses = tsk.mlp_train(net, x, T, 3000, 1e-3)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.25 * losses[0], (losses[0], losses[-1])

    hold = W.learned_holdout()
    hops = [_kop(tsk, c) for c in hold]
    m, k, tol = hold[0]["m"], hold[0]["k"], hold[0]["tol"]
    exact = [_fold(_exact_top(c, k)) for c in hold]
    n_rand, n_learn = [], []
    for seed in range(3):
        seeds = [100 * seed + i for i in range(len(hold))]
        rr = tsk.batch_arnoldi(hops, m, k, tol, seeds=seeds)
        v0s = []
        for c, op, s in zip(hold, hops, seeds):
            v, used = tsk.mlp_start(net, op, c["Re"], c["alpha"], GAMMA, s)
            assert used
            v0s.append(v)
        rl = tsk.batch_arnoldi(hops, m, k, tol, v0s=v0s)
        for i, (a, b) in enumerate(zip(rr, rl)):
            assert b["status"] == tsk.TSK_OK, (seed, i)        # the learned start always converged
            assert match_sets(_fold(b["lam"]), exact[i]) <= FP32_LAMBDA_BOUND, (seed, i)
            if a["status"] == tsk.TSK_OK:
                assert match_sets(_fold(a["lam"]), exact[i]) <= FP32_LAMBDA_BOUND, (seed, i)
            n_rand.append(a["n_matvec"])
            n_learn.append(b["n_matvec"])
    print(f"\nheld-out mean matvecs to {k} pairs: random {np.mean(n_rand):.2f}, learned {np.mean(n_learn):.2f}")
    assert np.mean(n_learn) <= 0.9 * np.mean(n_rand), (np.mean(n_rand), np.mean(n_learn))
