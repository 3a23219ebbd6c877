"""GPU parity of the general two-dimensional base-flow path (full 2-D
pseudo-spectral pipeline) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.kolmogorov import Kolmogorov, base_from_streamfunction

pytestmark = pytest.mark.gpu


def _general(tsk, N, alpha=0.5, Re=20.0, dt=0.005, T=1.0, prec=0, seed=0, fields=None):
    if fields is None:
        fields = base_from_streamfunction(W.random_base_modes(2, seed), N, alpha)
    U, V, Ox, Oy = fields
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    tsk.set_base_flow(op, U, V, Ox, Oy)
    return op, Kolmogorov(N, alpha, Re, dt, T, U, V, Ox, Oy)


def _phys(op, a):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda().reshape(-1)


def _to_phys(tsk, op, state):
    out = torch.zeros(op.N * op.N, dtype=state.dtype, device="cuda")
    tsk.to_physical(op, state, out)
    return out.double().cpu().numpy().reshape(op.N, op.N)


@pytest.mark.parametrize("N,T,prec", [(16, 1.0, 0), (48, 0.5, 0), (64, 0.2, 0), (96, 0.05, 0), (128, 0.05, 0),
                                      (384, 0.005, 0), (128, 0.1, 1), (512, 0.005, 1)])
def test_general_matvec_matches_oracle(tsk, N, T, prec):
    print(f"general base matvec N={N} T={T} prec={prec}", flush=True)
    op, ref = _general(tsk, N, T=T, prec=prec, seed=N)
    w = ref.project(W.kolmo_start_physical(N, 5))
    x = op.new_state()
    tsk.from_physical(op, _phys(op, w), x)
    y = op.new_state()
    tsk.apply(op, x, y)
    got = _to_phys(tsk, op, y)
    want = ref.apply(w)
    tol = 1e-11 if prec == 0 else 2e-5
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want)), np.max(np.abs(got - want)) / np.max(np.abs(want))


def test_general_path_reduces_to_the_column_stepper_for_a_parallel_base(tsk):
    N, alpha = 128, 0.5
    y = 2 * np.pi * np.arange(N) / N
    Ug = np.repeat(np.sin(4 * y)[:, None], N, axis=1)
    Oyg = np.repeat((16 * np.sin(4 * y))[:, None], N, axis=1)
    z = np.zeros((N, N))
    print("general base = Kolmogorov base, N=128 T=1", flush=True)
    op, _ = _general(tsk, N, alpha, fields=(Ug, z, z, Oyg))
    col = tsk.create_kolmo2d(N, 0)
    tsk.set_params_kolmo(col, 20.0, alpha, 0.005, 1.0)
    tsk.set_base_kolmogorov(col, 4)
    x = col.new_state()
    tsk.from_physical(col, _phys(col, W.kolmo_start_physical(N, 6)), x)
    a, b = op.new_state(), col.new_state()
    tsk.apply(op, x, a)
    tsk.apply(col, x, b)
    assert torch.max(torch.abs(a - b)).item() <= 1e-12 * torch.max(torch.abs(b)).item()


@pytest.mark.parametrize("N", [32, 48])
def test_general_arnoldi_same_steps_and_ritz_values(tsk, N):
    print(f"general base arnoldi N={N}", flush=True)
    op, ref = _general(tsk, N, seed=100 + N)
    w0 = W.kolmo_start_physical(N, 7)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, w0), x)
    r = tsk.arnoldi(op, 40, 6, 1e-8, v0=x)
    o = oracle_arnoldi(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), 40, 6, 1e-8,
                       T=ref.T)
    assert r["status"] == o["status"]
    assert abs(r["n_matvec"] - o["n_matvec"]) <= 1
    # the last wanted value may be either member of a conjugate pair (equal |mu|)
    fold = lambda lam: np.array([complex(z.real, abs(z.imag)) for z in lam])
    assert match_sets(fold(r["lam"]), fold(o["lam"])) <= 1e-8


def test_batch_with_general_and_parallel_operators_equals_single_runs(tsk):
    N = 32
    g, _ = _general(tsk, N, seed=3)
    p = tsk.create_kolmo2d(N, 0)
    tsk.set_params_kolmo(p, 20.0, 0.5, 0.005, 1.0)
    tsk.set_base_kolmogorov(p, 4)
    singles = [tsk.arnoldi(op, 30, 4, 1e-8, seed=11 + i) for i, op in enumerate((g, p))]
    batch = tsk.batch_arnoldi([g, p], 30, 4, 1e-8, seeds=[11, 12])
    for s, b in zip(singles, batch):
        assert s["n_matvec"] == b["n_matvec"] and s["status"] == b["status"]
        assert np.array_equal(s["lam"], b["lam"])


def test_general_base_validation_and_switch_back(tsk):
    N = 16
    op = tsk.create_kolmo2d(N, 0)
    tsk.set_params_kolmo(op, 20.0, 0.5, 0.005, 1.0)
    U, V, Ox, Oy = base_from_streamfunction(W.random_base_modes(2, 1), N, 0.5)
    bad = U.copy()
    bad[3, 4] = np.nan
    with pytest.raises(tsk.TskError) as e:
        tsk.set_base_flow(op, bad, V, Ox, Oy)
    assert e.value.status == tsk.TSK_ENONFINITE
    tsk.set_base_flow(op, U, V, Ox, Oy)
    tsk.set_base_kolmogorov(op, 4)          # back to the column stepper
    ref = Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.005, 1.0, 4)
    w = ref.project(W.kolmo_start_physical(N, 8))
    x, y = op.new_state(), op.new_state()
    tsk.from_physical(op, _phys(op, w), x)
    tsk.apply(op, x, y)
    want = ref.apply(w)
    assert np.max(np.abs(_to_phys(tsk, op, y) - want)) <= 1e-11 * np.max(np.abs(want))
