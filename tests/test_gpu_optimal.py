"""GPU parity of the adjoint propagators and of the optimal perturbation (Lanczos
on M^dagger M; Sec. 2.3.1 SVD formulation, Sec. 3.3.2) against the CPU oracle,
through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.cgle import CGLE
from oracle.kolmogorov import Kolmogorov, base_from_streamfunction
from oracle.optimal import cgle_apply_adjoint, kolmo_apply_adjoint, optimal_perturbation

pytestmark = pytest.mark.gpu


def _op(tsk, N, alpha=0.5, Re=20.0, dt=0.005, T=1.0, prec=0, base="kolmogorov"):
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    if base == "general":  # random band-limited 2-D base: the transposed 2-D pipeline
        U, V, Ox, Oy = base_from_streamfunction(W.random_base_modes(2, 1), N, alpha)
        tsk.set_base_flow(op, U, V, Ox, Oy)
        return op, Kolmogorov(N, alpha, Re, dt, T, U, V, Ox, Oy)
    if base in ("kolmogorov", "kolmogorov-columns"):
        tsk.set_base_kolmogorov(op, 4)
        if base == "kolmogorov-columns":  # the transposed column stepper instead of the coupling one
            tsk.set_tuning(op, 1)
        return op, Kolmogorov.kolmogorov(N, alpha, Re, dt, T, 4)
    y = 2 * np.pi * np.arange(N) / N
    if base == "shifted":  # one harmonic with a phase: the coupling steppers with y0 != 0
        U = 0.8 * np.sin(4 * (y - 0.3))
        dO = 16.0 * U  # -U''
    else:
        U = np.sin(y) + 0.5 * np.cos(2 * y)
        dO = np.sin(y) + 2.0 * np.cos(2 * y)  # -U''
    tsk.set_base_parallel(op, U, dO)
    Ug = np.repeat(U[:, None], N, axis=1)
    Og = np.repeat(dO[:, None], N, axis=1)
    z = np.zeros((N, N))
    return op, Kolmogorov(N, alpha, Re, dt, T, Ug, z, z, Og)


def _state(tsk, op, w):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    x = op.new_state()
    tsk.from_physical(op, torch.from_numpy(np.ascontiguousarray(w)).to(dt).cuda().reshape(-1), x)
    return x


def _phys(tsk, op, s):
    out = torch.zeros(op.N * op.N, dtype=s.dtype, device="cuda")
    tsk.to_physical(op, s, out)
    return out.double().cpu().numpy().reshape(op.N, op.N)


@pytest.mark.parametrize("N,T,base,prec", [(16, 1.0, "kolmogorov", 0), (48, 0.5, "kolmogorov", 0),
                                           (48, 0.5, "parallel", 0), (128, 1.0, "kolmogorov", 0),
                                           (128, 0.1, "parallel", 0), (128, 0.1, "kolmogorov-columns", 0),
                                           (128, 0.5, "shifted", 0), (384, 0.01, "kolmogorov", 0),
                                           (512, 0.01, "parallel", 0), (512, 0.1, "kolmogorov", 0),
                                           (128, 0.1, "kolmogorov", 1), (256, 0.1, "shifted", 1),
                                           (512, 0.01, "kolmogorov", 1), (16, 1.0, "general", 0),
                                           (48, 0.5, "general", 0), (128, 0.1, "general", 0),
                                           (384, 0.01, "general", 0), (96, 0.2, "general", 1),
                                           (512, 0.01, "general", 1)])
def test_adjoint_matvec_matches_oracle(tsk, N, T, base, prec):
    # kolmogorov and shifted: the transposed spectral-coupling stepper (512: two
    # modes per lane); parallel and kolmogorov-columns: the transposed column
    # stepper; general: the transposed 2-D pipeline
    print(f"adjoint matvec N={N} T={T} base={base} prec={prec}", flush=True)
    op, ref = _op(tsk, N, T=T, prec=prec, base=base)
    assert tsk.get_tuning(op) == (-2 if base in ("kolmogorov", "shifted") else 1 if base == "kolmogorov-columns"
                                  else tsk.get_tuning(op))
    z = ref.project(W.kolmo_start_physical(N, 5))
    x = _state(tsk, op, z)
    y = op.new_state()
    tsk.apply_adjoint(op, x, y)
    got = _phys(tsk, op, y)
    want = kolmo_apply_adjoint(ref, z)
    tol = 1e-11 if prec == 0 else 2e-5
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


@pytest.mark.parametrize("N,base", [(128, "kolmogorov"), (128, "parallel"), (128, "shifted"), (512, "kolmogorov"),
                                    (128, "general"), (48, "general")])
def test_device_adjoint_satisfies_the_dot_product_identity(tsk, N, base):
    print(f"adjoint dot product N={N} base={base}", flush=True)
    op, ref = _op(tsk, N, base=base)
    x = _state(tsk, op, W.kolmo_start_physical(N, 1))
    y = _state(tsk, op, W.kolmo_start_physical(N, 2))
    Mx, Mty = op.new_state(), op.new_state()
    tsk.apply(op, x, Mx)
    tsk.apply_adjoint(op, y, Mty)
    lhs, rhs = torch.dot(Mx, y).item(), torch.dot(x, Mty).item()
    assert abs(lhs - rhs) <= 1e-12 * torch.linalg.norm(Mx).item() * torch.linalg.norm(y).item()


def test_cgle_adjoint_matches_oracle(tsk):
    print("adjoint cgle", flush=True)
    ref = CGLE()
    op = tsk.create_cgle1d(256)
    tsk.set_params_cgle(op, 2.0, 0.2, -1.0, 0.41, -0.01, 0.01, 1.0)
    u = W.cgle_start(256, 4)
    x = torch.from_numpy(u).cuda()
    y = torch.zeros_like(x)
    tsk.apply_adjoint(op, x, y)
    want = cgle_apply_adjoint(ref, u)
    assert np.max(np.abs(y.cpu().numpy() - want)) <= 1e-12 * np.max(np.abs(want))
    # <M a, b> = <a, M^H b>
    a, b = torch.from_numpy(W.cgle_start(256, 5)).cuda(), torch.from_numpy(W.cgle_start(256, 6)).cuda()
    Ma, Mhb = torch.zeros_like(a), torch.zeros_like(b)
    tsk.apply(op, a, Ma)
    tsk.apply_adjoint(op, b, Mhb)
    lhs, rhs = torch.vdot(Ma, b).item(), torch.vdot(a, Mhb).item()
    assert abs(lhs - rhs) <= 1e-12 * torch.linalg.norm(Ma).item() * torch.linalg.norm(b).item()


@pytest.mark.parametrize("N,base", [(32, "kolmogorov"), (48, "parallel"), (32, "general")])
def test_optimal_perturbation_matches_oracle(tsk, N, base):
    print(f"optimal perturbation N={N} base={base}", flush=True)
    op, ref = _op(tsk, N, base=base)
    w0 = ref.project(W.kolmo_start_physical(N, 0))
    r = tsk.optimal_perturbation(op, 40, 3, 1e-9, v0=_state(tsk, op, w0), want_vectors=True)
    o = optimal_perturbation(lambda v: ref.apply(v.reshape(N, N)).ravel(),
                             lambda v: kolmo_apply_adjoint(ref, v.reshape(N, N)).ravel(), w0.ravel(), 40, 3, 1e-9)
    assert r["status"] == o["status"] == 0
    assert abs(r["n_steps"] - o["n_steps"]) <= 1
    assert np.max(np.abs(np.sort(r["sigma"]) - np.sort(o["sigma"]))) <= 1e-10 * np.max(o["sigma"])
    assert np.all(r["res"] <= 1e-9)
    # optimal initial condition: ||M x|| = sigma, and M^dagger M x = sigma^2 x
    for sig, xv in zip(r["sigma"], r["X"]):
        x = xv.real.contiguous()
        assert torch.max(torch.abs(xv.imag)).item() == 0.0
        Mx, MtMx = op.new_state(), op.new_state()
        tsk.apply(op, x, Mx)
        tsk.apply_adjoint(op, Mx, MtMx)
        assert abs(torch.linalg.norm(Mx).item() - sig) <= 1e-9 * sig
        assert torch.linalg.norm(MtMx - sig * sig * x).item() <= 1e-8 * sig * sig


def test_cgle_optimal_perturbation_matches_oracle(tsk):
    print("optimal perturbation cgle", flush=True)
    ref = CGLE()
    op = tsk.create_cgle1d(256)
    tsk.set_params_cgle(op, 2.0, 0.2, -1.0, 0.41, -0.01, 0.01, 1.0)
    u0 = W.cgle_start(256, 0)
    r = tsk.optimal_perturbation(op, 40, 2, 1e-10, v0=torch.from_numpy(u0).cuda())
    o = optimal_perturbation(ref.apply, lambda v: cgle_apply_adjoint(ref, v), u0, 40, 2, 1e-10)
    assert r["status"] == o["status"] == 0
    assert r["n_steps"] == o["n_steps"]
    assert np.max(np.abs(np.sort(r["sigma"]) - np.sort(o["sigma"]))) <= 1e-10 * np.max(o["sigma"])


def test_full_size_gain_bounds_and_fp32_form(tsk):
    # 128^2 (the benchmark operator): sigma_1 = ||M|| >= the spectral radius, the
    # optimal initial condition attains it, and the FP32 form agrees to 1e-5
    N = 128
    print("optimal perturbation N=128 fp64 and fp32", flush=True)
    op, _ = _op(tsk, N)
    op32, _ = _op(tsk, N, prec=1)
    r = tsk.optimal_perturbation(op, 40, 2, 1e-8, seed=0, want_vectors=True)
    a = tsk.arnoldi(op, 64, 1, 1e-8, seed=0)
    assert r["status"] == 0 and a["status"] == 0
    assert r["sigma"][0] >= abs(a["mu"][0]) * (1 - 1e-12)
    x = r["X"][0].real.contiguous()
    Mx = op.new_state()
    tsk.apply(op, x, Mx)
    assert abs(torch.linalg.norm(Mx).item() - r["sigma"][0]) <= 1e-9 * r["sigma"][0]
    r32 = tsk.optimal_perturbation(op32, 40, 2, 1e-8, seed=0)
    assert r32["status"] == 0
    assert abs(r32["sigma"][0] - r["sigma"][0]) <= 1e-5 * r["sigma"][0]


def test_adjoint_argument_errors_are_rejected(tsk):
    print("adjoint validation", flush=True)
    N = 32
    op, _ = _op(tsk, N, base="general")
    x = op.new_state()
    with pytest.raises(tsk.TskError):  # aliasing
        tsk.apply_adjoint(op, x, x)
    op2, _ = _op(tsk, N)
    with pytest.raises(tsk.TskError):
        tsk.apply_adjoint(op2, x, x)
    op3 = tsk.create_kolmo2d(N, 0)  # no parameters or base flow yet
    y = op3.new_state()
    with pytest.raises(tsk.TskError):
        tsk.apply_adjoint(op3, x, y)
