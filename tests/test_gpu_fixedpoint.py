"""GPU parity of the nonlinear stepper and of the fixed-point solvers (Sec. 3.1:
selective frequency damping, recursive projection method, BoostConv) against the
CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.fixedpoint import NonlinearKolmogorov, boostconv, rpm, sfd, unstable_basis

pytestmark = pytest.mark.gpu


def _pair(tsk, N, Re=7.0, dt=0.02, T=2.0, U0=0.7, amp=0.002, prec=0, seed=7):
    ex = W.random_forcing_field(N, 0.5, 2, seed, amp) if amp > 0 else None
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, 0.5, dt, T)
    tsk.set_base_kolmogorov(op, 4)
    tsk.set_nonlinear(op, 4, U0, ex)
    return op, NonlinearKolmogorov(N, 0.5, Re, dt, T, U0=U0, extra_forcing=ex)


def _state(tsk, op, w):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    x = op.new_state()
    tsk.from_physical(op, torch.from_numpy(np.ascontiguousarray(w)).to(dt).cuda().reshape(-1), x)
    return x


def _phys(tsk, op, s):
    out = torch.zeros(op.N * op.N, dtype=s.dtype, device="cuda")
    tsk.to_physical(op, s, out)
    return out.double().cpu().numpy().reshape(op.N, op.N)


@pytest.mark.parametrize("N,T,prec", [(16, 0.4, 0), (48, 0.2, 0), (128, 0.05, 0), (256, 0.02, 0), (128, 0.05, 1)])
def test_nonlinear_step_matches_oracle(tsk, N, T, prec):
    print(f"nonlinear step N={N} T={T} prec={prec}", flush=True)
    op, ref = _pair(tsk, N, Re=20.0, dt=0.005 if N > 48 else 0.02, T=T, amp=0.05, prec=prec)
    w = ref.omega_lam + ref.lin.project(W.random_forcing_field(N, 0.5, 3, 11, 0.2))
    x, y = _state(tsk, op, w), op.new_state()
    tsk.nonlinear_step(op, x, y, 0)
    got = _phys(tsk, op, y)
    want = ref.apply(w)
    tol = 1e-11 if prec == 0 else 2e-5
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


def test_laminar_state_is_a_fixed_point_on_the_device(tsk):
    print("laminar fixed point N=64", flush=True)
    op, ref = _pair(tsk, 64, Re=20.0, dt=0.005, T=1.0, amp=0.0)
    lam = tsk.laminar_state(op)
    assert np.max(np.abs(_phys(tsk, op, lam) - ref.omega_lam)) <= 1e-13 * 4
    y = op.new_state()
    tsk.nonlinear_step(op, lam, y, 0)
    assert torch.max(torch.abs(y - lam)).item() <= 1e-12 * torch.max(torch.abs(lam)).item()


def test_base_from_state_is_the_oracle_linearization(tsk):
    N = 48
    print(f"base from state N={N}", flush=True)
    op, ref = _pair(tsk, N, Re=20.0, dt=0.01, T=0.2, amp=0.05)
    w = ref.omega_lam + ref.lin.project(W.random_forcing_field(N, 0.5, 2, 12, 0.3))
    tsk.set_base_from_state(op, _state(tsk, op, w))
    v = ref.lin.project(W.kolmo_start_physical(N, 3))
    y = op.new_state()
    tsk.apply(op, _state(tsk, op, v), y)
    want = ref.linearized_about(w).apply(v)
    assert np.max(np.abs(_phys(tsk, op, y) - want)) <= 1e-11 * np.max(np.abs(want))


# The device state's Euclidean norm is the RMS of the physical field, the
# oracle's the grid sum: ||.||_oracle = N ||.||_device for the same field, so
# tolerances and residual histories convert by the factor N.
def _oracle_problem(ref, N):
    G = lambda v: ref.apply(v.reshape(N, N)).ravel()
    return G, ref.omega_lam.ravel().copy()


@pytest.mark.parametrize("N", [16, 32])
def test_rpm_matches_oracle_and_the_fixed_point_is_then_the_base_flow(tsk, N):
    print(f"rpm N={N}", flush=True)
    op, ref = _pair(tsk, N)
    x = tsk.laminar_state(op)
    r = tsk.rpm(op, x, 24, 1, 0.3, 1e-8, 60)
    G, x0 = _oracle_problem(ref, N)
    lin = ref.linearized_about(x0.reshape(N, N))
    U, H, kept = unstable_basis(lambda v: lin.apply(v.reshape(N, N)).ravel(), G(x0) - x0, 24, 1, 0.3)
    xo, ho, ito = rpm(G, x0, U, H, 1e-8 * N, 60)
    assert r["status"] == 0 and r["basis_dim"] == U.shape[1]
    assert abs(r["iterations"] - ito) <= 2
    got = _phys(tsk, op, x).ravel()
    assert np.linalg.norm(got - xo) <= 1e-7 * np.linalg.norm(xo)
    n = min(len(r["hist"]), len(ho), 8)
    assert np.max(np.abs(N * r["hist"][:n] - ho[:n]) / ho[:n]) <= 1e-5
    # the operator is now linearized about the fixed point: its eigenvalues
    a = tsk.arnoldi(op, 40, 4, 1e-9, seed=1)
    lin_fp = ref.linearized_about(xo.reshape(N, N))
    o = oracle_arnoldi(lambda v: lin_fp.apply(v.reshape(N, N)).ravel(),
                       lin_fp.project(W.kolmo_start_physical(N, 1)).ravel(), 40, 4, 1e-9, T=ref.T)
    fold = lambda lam: np.array([complex(z.real, abs(z.imag)) for z in lam])
    assert a["status"] == 0 and o["status"] == 0
    assert match_sets(fold(a["lam"]), fold(o["lam"])) <= 1e-6


def test_boostconv_matches_oracle(tsk):
    N = 16
    print(f"boostconv N={N}", flush=True)
    op, ref = _pair(tsk, N)
    x = tsk.laminar_state(op)
    r = tsk.boostconv(op, x, 10, 1e-9, 80)
    G, x0 = _oracle_problem(ref, N)
    conds = []
    xo, ho, ito = boostconv(G, x0, 10, 1e-9 * N, 80, conds=conds)
    # The device solves for c = Y^+ r by the normal equations, the oracle by an
    # SVD least-squares solve: they differ by about cond(Y)^2 u per iteration.
    # With cond(Y) <= 1e4 along the run that is <= 1e-8, far below the 1e-5 bar
    # on the residual histories (which also carry the stepper's 1e-11).
    assert max(conds) <= 1e4, max(conds)
    assert r["status"] == 0
    assert abs(r["iterations"] - ito) <= 3
    got = _phys(tsk, op, x).ravel()
    assert np.linalg.norm(got - xo) <= 1e-7 * np.linalg.norm(xo)
    n = min(len(r["hist"]), len(ho))
    big = ho[:n] >= 1e-6   # well above the tolerance, where relative deviations are meaningful
    assert np.max(np.abs(N * r["hist"][:n] - ho[:n])[big] / ho[:n][big]) <= 1e-5


def test_sfd_matches_oracle(tsk):
    N = 16
    print(f"sfd N={N}", flush=True)
    op, ref = _pair(tsk, N)
    x = tsk.laminar_state(op)
    r = tsk.sfd(op, x, 0.2, 5.0, 100, 1e-5, 80)
    step = lambda v: ref.lin.to_physical(ref.step_hat(ref.lin.to_spectral(v.reshape(N, N)))).ravel()
    xo, ho, so = sfd(step, ref.omega_lam.ravel(), 0.2, 5.0, ref.dt, 100, 1e-5 * N, 80)
    assert r["status"] == 0
    assert r["iterations"] == len(ho)
    got = _phys(tsk, op, x).ravel()
    assert np.linalg.norm(got - xo) <= 1e-8 * np.linalg.norm(xo)
    assert np.max(np.abs(N * r["hist"] - ho) / ho) <= 1e-6


def test_solvers_agree_on_the_device_and_fp32_form(tsk):
    N = 32
    print(f"solvers agree N={N} fp64 and fp32", flush=True)
    op, ref = _pair(tsk, N)
    xr = tsk.laminar_state(op)
    tsk.rpm(op, xr, 24, 1, 0.3, 1e-9, 80)
    xb = tsk.laminar_state(op)
    tsk.boostconv(op, xb, 10, 1e-9, 80)
    assert torch.linalg.norm(xr - xb).item() <= 1e-7 * torch.linalg.norm(xr).item()
    op32, _ = _pair(tsk, N, prec=1)
    x32 = tsk.laminar_state(op32)
    r32 = tsk.boostconv(op32, x32, 10, 1e-5, 80)
    assert r32["status"] == 0
    assert torch.linalg.norm(x32.double() - xr).item() <= 1e-4 * torch.linalg.norm(xr).item()


def test_validation(tsk):
    print("fixed-point validation", flush=True)
    op = tsk.create_kolmo2d(32, 0)
    tsk.set_params_kolmo(op, 7.0, 0.5, 0.02, 2.0)
    tsk.set_base_kolmogorov(op, 4)
    x, y = op.new_state(), op.new_state()
    with pytest.raises(tsk.TskError):
        tsk.nonlinear_step(op, x, y)   # nonlinear equation not set
    with pytest.raises(tsk.TskError):
        tsk.set_nonlinear(op, 11, 0.0)  # forcing wavenumber beyond (N-1)/3
    tsk.set_nonlinear(op, 4, 0.0)
    with pytest.raises(tsk.TskError):
        tsk.nonlinear_step(op, x, x)   # aliasing
    with pytest.raises(tsk.TskError):
        tsk.rpm(op, x, 3, 2, 0.1, 1e-8, 10)  # m < k + 2
    with pytest.raises(tsk.TskError):
        tsk.sfd(op, x, -1.0, 1.0, 10, 1e-8, 10)
    cg = tsk.create_cgle1d(64)
    tsk.set_params_cgle(cg, 2.0, 0.2, -1.0, 0.41, -0.01, 0.01, 1.0)
    z = torch.zeros(64, dtype=torch.complex128, device="cuda")
    with pytest.raises(tsk.TskError):
        tsk.boostconv(cg, z, 5, 1e-8, 10)
