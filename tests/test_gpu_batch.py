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


def test_neutral_curve_sweep_full_size(tsk):
    # 64 instances (24 x 128^2, 20 x 256^2, 20 x 384^2), FP32, m = 64, k = 4.
    print("batch sweep 64 instances", flush=True)
    sweep = W.batch_sweep(64, 0)
    ops = [_kolmo(tsk, c["N"], c["Re"], c["alpha"], 1) for c in sweep]
    rb = tsk.batch_arnoldi(ops, 64, 4, 1e-8, seeds=list(range(64)))
    assert all(b["status"] >= 0 for b in rb)
    # leading eigenvalue of a sample of instances against dense Galerkin blocks
    for i in (0, 1, 5, 10, 30, 63):
        c = sweep[i]
        blocks = galerkin_sinusoidal_blocks(c["N"], c["alpha"], c["Re"])
        lead = max(np.max(np.linalg.eigvals(A).real) for _, A in blocks.values())
        got = np.max(rb[i]["lam"].real)
        assert abs(got - lead) <= 2e-5, (i, got, lead)
