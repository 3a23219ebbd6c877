"""Batched Arnoldi (neutral-curve sweep): a batch advances instances in lockstep
with shared launches; every instance must give exactly what it gives alone."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.kolmogorov import Kolmogorov, galerkin_sinusoidal_blocks

pytestmark = pytest.mark.gpu


def _kolmo(tsk, N, Re, alpha, prec=0):
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, 0.005, 1.0)
    tsk.set_base_kolmogorov(op, 4)
    return op


def _start(tsk, op, N, seed):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    x = op.new_state()
    tsk.from_physical(op, torch.from_numpy(W.kolmo_start_physical(N, seed)).to(dt).cuda().reshape(-1), x)
    return x


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_single_runs_bitwise(tsk, prec):
    print(f"batch vs single prec={prec}", flush=True)
    cfg = [(32, 20.0, 0.5), (48, 12.0, 0.75), (48, 30.0, 1.0), (64, 25.0, 0.25)]
    ops = [_kolmo(tsk, N, Re, a, prec) for N, Re, a in cfg]
    v0s = [_start(tsk, op, N, i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    rb = tsk.batch_arnoldi(ops, 40, 4, 1e-8, v0s=v0s, want_vectors=True)
    for op, v0, b in zip(ops, v0s, rb):
        r = tsk.arnoldi(op, 40, 4, 1e-8, v0=v0, want_vectors=True)
        assert b["status"] == r["status"] and b["n_matvec"] == r["n_matvec"]
        assert np.array_equal(b["lam"], r["lam"]) and np.array_equal(b["res"], r["res"])
        assert torch.equal(b["X"], r["X"])


@pytest.mark.parametrize("prec", [0, 1])
def test_bloch_sector_batch_equals_single_runs_bitwise(tsk, prec):
    # 128^2 and 256^2 Kolmogorov instances take the Bloch-sector stepper alone
    # and in a batch (one launch per grid size, instances on grid y); the 48^2
    # one takes the column stepper in its own group
    print(f"bloch batch vs single prec={prec}", flush=True)
    cfg = [(128, 20.0, 0.5), (256, 12.0, 0.75), (128, 30.0, 1.0), (48, 25.0, 0.25)]
    ops = [_kolmo(tsk, N, Re, a, prec) for N, Re, a in cfg]
    for op in ops[:3]:
        tsk.set_tuning(op, 3)   # Bloch sectors instead of the default coupling stepper
    tsk.set_tuning(ops[3], 1)
    assert [tsk.get_tuning(op) for op in ops] == [-1, -1, -1, 1]
    v0s = [_start(tsk, op, N, i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    rb = tsk.batch_arnoldi(ops, 40, 4, 1e-8, v0s=v0s, want_vectors=True)
    for op, v0, b in zip(ops, v0s, rb):
        r = tsk.arnoldi(op, 40, 4, 1e-8, v0=v0, want_vectors=True)
        assert b["status"] == r["status"] and b["n_matvec"] == r["n_matvec"]
        assert np.array_equal(b["lam"], r["lam"]) and np.array_equal(b["res"], r["res"])
        assert torch.equal(b["X"], r["X"])


def test_bloch_sector_batch_512_equals_single_runs_bitwise(tsk):
    # 512^2 FP32: 128-mode sectors, two modes per lane, in a batched launch
    print("bloch batch 512 vs single", flush=True)
    cfg = [(512, 20.0, 0.5), (512, 30.0, 1.0), (128, 15.0, 0.75)]
    ops = [_kolmo(tsk, N, Re, a, 1) for N, Re, a in cfg]
    for op in ops:
        tsk.set_tuning(op, 3)
    assert [tsk.get_tuning(op) for op in ops] == [-1, -1, -1]
    v0s = [_start(tsk, op, N, 10 + i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    rb = tsk.batch_arnoldi(ops, 24, 2, 1e-6, v0s=v0s, want_vectors=True)
    for op, v0, b in zip(ops, v0s, rb):
        r = tsk.arnoldi(op, 24, 2, 1e-6, v0=v0, want_vectors=True)
        assert b["status"] == r["status"] and b["n_matvec"] == r["n_matvec"]
        assert np.array_equal(b["lam"], r["lam"]) and np.array_equal(b["res"], r["res"])
        assert torch.equal(b["X"], r["X"])


@pytest.mark.parametrize("prec", [0, 1])
def test_coupling_stepper_batch_of_mixed_sizes_equals_single_runs_bitwise(tsk, prec):
    # the one-harmonic base takes the spectral-coupling stepper at every grid size,
    # and a batch runs all of them in one launch (instances on grid y)
    print(f"coupling batch vs single prec={prec}", flush=True)
    cfg = [(128, 20.0, 0.5), (384, 12.0, 0.75), (256, 30.0, 1.0), (48, 25.0, 0.25), (512, 8.0, 0.5)]
    ops = [_kolmo(tsk, N, Re, a, prec) for N, Re, a in cfg]
    assert [tsk.get_tuning(op) for op in ops] == [-2] * len(ops)
    v0s = [_start(tsk, op, N, 20 + i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    rb = tsk.batch_arnoldi(ops, 40, 4, 1e-8, v0s=v0s, want_vectors=True)
    for op, v0, b in zip(ops, v0s, rb):
        r = tsk.arnoldi(op, 40, 4, 1e-8, v0=v0, want_vectors=True)
        assert b["status"] == r["status"] and b["n_matvec"] == r["n_matvec"]
        assert np.array_equal(b["lam"], r["lam"]) and np.array_equal(b["res"], r["res"])
        assert torch.equal(b["X"], r["X"])


@pytest.mark.parametrize("prec", [0, 1])
def test_coupling_stepper_launch_shapes_agree_bitwise(tsk, prec):
    # 1, 2 or 4 wavefronts per workgroup (the tuned launch shape): the same bits,
    # alone and in a batch; the tuned choice is one of them
    print(f"coupling launch shapes prec={prec}", flush=True)
    cfg = [(128, 20.0, 0.5), (384, 12.0, 0.75), (512, 30.0, 1.0)]
    ops = [_kolmo(tsk, N, Re, a, prec) for N, Re, a in cfg]
    for op, (N, _, _) in zip(ops, cfg):
        x = _start(tsk, op, N, 7)
        outs = []
        for w in (1, 2, 4):
            tsk.set_stepper_waves(op, w)
            assert tsk.get_stepper_waves(op) == w
            y = op.new_state()
            tsk.apply(op, x, y)
            outs.append(y)
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
        tsk.set_stepper_waves(op, 0)
        y = op.new_state()
        tsk.apply(op, x, y)
        assert torch.equal(y, outs[0]) and tsk.get_stepper_waves(op) in (1, 2, 4)
    with pytest.raises(tsk.TskError):
        tsk.set_stepper_waves(ops[0], 3)
    v0s = [_start(tsk, op, N, 40 + i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    res = []
    for w in (1, 4):
        for op in ops:
            tsk.set_stepper_waves(op, w)
        res.append(tsk.batch_arnoldi(ops, 20, 2, 1e-8, v0s=v0s))
    for a, b in zip(*res):
        assert a["n_matvec"] == b["n_matvec"] and np.array_equal(a["lam"], b["lam"])


def test_batch_member_matches_oracle(tsk):
    print("batch member vs oracle", flush=True)
    cfg = [(48, 20.0, 0.5), (32, 10.0, 1.0)]
    ops = [_kolmo(tsk, N, Re, a) for N, Re, a in cfg]
    v0s = [_start(tsk, op, N, 3) for op, (N, _, _) in zip(ops, cfg)]
    rb = tsk.batch_arnoldi(ops, 40, 4, 1e-8, v0s=v0s)
    for (N, Re, a), b in zip(cfg, rb):
        ref = Kolmogorov.kolmogorov(N, a, Re, 0.005, 1.0, 4)
        o = oracle_arnoldi(lambda v: ref.apply(v.reshape(N, N)).ravel(),
                           ref.project(W.kolmo_start_physical(N, 3)).ravel(), 40, 4, 1e-8, T=1.0)
        assert b["n_matvec"] == o["n_matvec"]
        assert match_sets(b["lam"], o["lam"]) <= 1e-8


def test_batch_of_ginzburg_landau_operators(tsk):
    print("batch cgle", flush=True)
    c = W.CGLE
    ops = []
    for mu0 in (0.41, 0.3):
        op = tsk.create_cgle1d(256, c["half_width"])
        tsk.set_params_cgle(op, c["U"], c["c_u"], c["c_d"], mu0, c["mu2"], c["dt"], c["T"])
        ops.append(op)
    v0s = [torch.from_numpy(W.cgle_start(256, i)).cuda() for i in range(2)]
    rb = tsk.batch_arnoldi(ops, 40, 4, 1e-8, v0s=v0s)
    for op, v0, b in zip(ops, v0s, rb):
        r = tsk.arnoldi(op, 40, 4, 1e-8, v0=v0)
        assert b["n_matvec"] == r["n_matvec"] and np.array_equal(b["lam"], r["lam"])


def test_batch_rejects_mixed_precision_and_duplicates(tsk):
    a = _kolmo(tsk, 32, 20.0, 0.5, 0)
    b = _kolmo(tsk, 32, 20.0, 0.5, 1)
    with pytest.raises(tsk.TskError) as e:
        tsk.batch_arnoldi([a, b], 10, 2, 1e-8)
    assert e.value.status == tsk.TSK_EINVAL
    with pytest.raises(tsk.TskError) as e:
        tsk.batch_arnoldi([a, a], 10, 2, 1e-8)
    assert e.value.status == tsk.TSK_EINVAL


def _galerkin_top(N, alpha, Re, count):
    """The `count` leading distinct eigenvalues (by real part) of the dense
    Galerkin blocks of the linearized Kolmogorov operator."""
    blocks = galerkin_sinusoidal_blocks(N, alpha, Re)
    ev = np.concatenate([np.linalg.eigvals(A) for _, A in blocks.values()])
    ev = ev[np.argsort(-ev.real)]
    out = []
    for z in ev:
        if all(abs(z - w) > 1e-9 for w in out):
            out.append(z)
        if len(out) == count:
            break
    return np.array(out)


def test_neutral_curve_sweep_full_size(tsk):
    # 64 instances (24 x 128^2, 20 x 256^2, 20 x 384^2), FP32, m = 64, k = 4, all
    # converged: the instances not converged at order m restart (Krylov-Schur)
    print("batch sweep 64 instances, batched Krylov-Schur", flush=True)
    sweep = W.batch_sweep(64, 0)
    ops = [_kolmo(tsk, c["N"], c["Re"], c["alpha"], 1) for c in sweep]
    rb = tsk.batch_krylov_schur(ops, 64, 4, 1e-8, delta=0.1, seeds=list(range(64)))
    assert [b["status"] for b in rb] == [0] * 64
    assert any(b["n_restarts"] > 0 for b in rb)
    # the leading Galerkin eigenvalues are converged in the grid: at 384^2 they equal
    # the 128^2 ones to rounding, so every instance is checked against its 128^2 blocks
    c9 = sweep[9]
    assert np.max(np.abs(_galerkin_top(384, c9["alpha"], c9["Re"], 6) -
                         _galerkin_top(128, c9["alpha"], c9["Re"], 6))) <= 1e-10
    for i, (c, b) in enumerate(zip(sweep, rb)):
        top = _galerkin_top(128, c["alpha"], c["Re"], 8)
        assert b["n_ritz"] == 4
        # every returned value is an eigenvalue, and the four are the leading four
        # (FP32 form, stated bound 2e-5) whenever the fourth is separated from the fifth
        for lam in b["lam"]:
            assert np.min(np.abs(top - lam)) <= 2e-5, (i, lam)
        if top[3].real - top[4].real > 1e-4:
            assert match_sets(b["lam"], top[:4]) <= 2e-5, (i, b["lam"], top[:4])
        if b["n_restarts"] > 0:
            assert b["n_matvec"] > 64


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_krylov_schur_restarts_small(tsk, prec):
    # m small enough that most instances restart: FP64 every returned value is a
    # Galerkin eigenvalue to 1e-8 with residual <= tol; instances that converge
    # before order m equal the plain batched Arnoldi run bitwise
    print(f"batched krylov-schur small prec={prec}", flush=True)
    cfg = [(32, 20.0, 0.5), (48, 12.0, 0.75), (48, 30.0, 0.25), (64, 25.0, 1.0), (32, 8.0, 0.25)]
    m, k = 14, 4
    ops = [_kolmo(tsk, N, Re, a, prec) for N, Re, a in cfg]
    v0s = [_start(tsk, op, N, 30 + i) for i, (op, (N, _, _)) in enumerate(zip(ops, cfg))]
    rk = tsk.batch_krylov_schur(ops, m, k, 1e-8, delta=0.1, v0s=v0s, want_vectors=True)
    ra = tsk.batch_arnoldi(ops, m, k, 1e-8, v0s=v0s, want_vectors=True)
    bar = 1e-8 if prec == 0 else 2e-5
    assert any(b["n_restarts"] > 0 for b in rk)
    for (N, Re, a), b, a_ in zip(cfg, rk, ra):
        assert b["status"] == 0
        assert np.all(b["res"] <= (1e-8 if prec == 0 else max(1e-8, 32 * 2.0 ** -24 * 2.0)))
        top = _galerkin_top(N, a, Re, 12)
        for lam in b["lam"]:
            assert np.min(np.abs(top - lam)) <= bar, (N, Re, a, lam)
        if a_["status"] == 0:
            assert b["n_restarts"] == 0 and b["n_matvec"] == a_["n_matvec"]
            assert np.array_equal(b["lam"], a_["lam"]) and torch.equal(b["X"], a_["X"])
        else:
            assert b["n_restarts"] >= 1 and b["n_matvec"] > m
            # Ritz vectors of the restarted instances: unit norm
            nrm = torch.linalg.norm(b["X"], dim=1).cpu().numpy()
            assert np.all(np.abs(nrm - 1.0) <= 1e-6)
