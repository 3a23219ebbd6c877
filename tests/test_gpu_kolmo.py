"""GPU parity of the linearized Navier-Stokes (Kolmogorov) path against the CPU
oracle, through the C ABI: physical <-> spectral transforms, the IF-RK4 matvec,
Arnoldi at small and full size."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.kolmogorov import Kolmogorov, galerkin_sinusoidal_blocks

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _op(tsk, N, alpha=0.5, Re=20.0, dt=0.005, T=1.0, prec=0, base="kolmogorov", U=None, dO=None):
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    if base == "kolmogorov":
        tsk.set_base_kolmogorov(op, 4)
        ref = Kolmogorov.kolmogorov(N, alpha, Re, dt, T, 4)
    else:
        tsk.set_base_parallel(op, U, dO)
        Ug = np.repeat(np.asarray(U)[:, None], N, axis=1)
        Og = np.repeat(np.asarray(dO)[:, None], N, axis=1)
        z = np.zeros((N, N))
        ref = Kolmogorov(N, alpha, Re, dt, T, Ug, z, z, Og)
    return op, ref


def _phys(op, N, a):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda().reshape(-1)


def _to_phys(tsk, op, state):
    out = torch.zeros(op.N * op.N, dtype=state.dtype, device="cuda")
    tsk.to_physical(op, state, out)
    return out.double().cpu().numpy().reshape(op.N, op.N)


@pytest.mark.parametrize("N", [16, 48, 128, 384, 512])
def test_transforms_project_like_the_oracle(tsk, N):
    print(f"kolmo transforms N={N}", flush=True)
    op, ref = _op(tsk, N)
    w = W.kolmo_start_physical(N, 2)
    s = op.new_state()
    tsk.from_physical(op, _phys(op, N, w), s)
    back = _to_phys(tsk, op, s)
    want = ref.project(w)
    assert np.max(np.abs(back - want)) <= 1e-12 * np.max(np.abs(want))
    # Euclidean norm of the state = RMS of the projected field
    assert abs(torch.linalg.norm(s).item() - np.sqrt(np.mean(want ** 2))) <= 1e-12 * np.sqrt(np.mean(want ** 2))


_ORACLE_MATVEC = {}


def _oracle_matvec(N, T):
    """The oracle's full rfft2 IF-RK4 matvec of the seeded projected field
    (cached: the FP64 and FP32 rows share it)."""
    if (N, T) not in _ORACLE_MATVEC:
        ref = Kolmogorov.kolmogorov(N, 0.5, 20.0, 0.005, T, 4)
        w = ref.project(W.kolmo_start_physical(N, 3))
        _ORACLE_MATVEC[(N, T)] = (w, ref.apply(w))
    return _ORACLE_MATVEC[(N, T)]


# (N, T, precision, stepper): stepper "auto" is the library's choice (for this
# one-harmonic base the spectral-coupling stepper, at every N: the kernel of the
# benchmark configurations), "bloch" forces the Bloch-sector stepper (128^2,
# 256^2, 512^2), "column" one kx column per wavefront of the FFT column stepper.
# Full T = 1 (200 IF-RK4 steps) at 128^2 and 256^2, 20 steps at 384^2 and 512^2.
# Bars: 1e-11 (FP64), 2e-5 (FP32 state, transforms and RK4) of max |M w|.
@pytest.mark.parametrize("N,T,prec,stepper", [
    (16, 1.0, 0, "auto"), (48, 1.0, 0, "auto"), (48, 1.0, 1, "auto"), (96, 0.05, 0, "auto"),
    (128, 1.0, 0, "auto"), (128, 1.0, 1, "auto"), (128, 1.0, 0, "bloch"), (128, 1.0, 1, "bloch"),
    (128, 0.1, 0, "column"), (128, 0.1, 1, "column"),
    (256, 1.0, 0, "auto"), (256, 1.0, 1, "auto"), (256, 1.0, 0, "bloch"), (256, 1.0, 1, "bloch"),
    (256, 1.0, 0, "column"),
    (384, 0.1, 0, "auto"), (384, 0.1, 1, "auto"), (384, 0.1, 1, "column"),
    (512, 0.1, 0, "auto"), (512, 0.1, 1, "auto"), (512, 0.1, 0, "bloch"), (512, 0.1, 1, "bloch"),
    (512, 0.1, 1, "column")])
def test_matvec_matches_oracle(tsk, N, T, prec, stepper):
    print(f"kolmo matvec N={N} T={T} prec={prec} stepper={stepper}", flush=True)
    op, _ = _op(tsk, N, T=T, prec=prec)
    expect = {"auto": -2, "bloch": -1, "column": 1}[stepper]
    tsk.set_tuning(op, {"auto": 0, "bloch": 3, "column": 1}[stepper])
    w, want = _oracle_matvec(N, T)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, w), x)
    y = op.new_state()
    tsk.apply(op, x, y)
    assert tsk.get_tuning(op) == expect
    got = _to_phys(tsk, op, y)
    tol = 1e-11 if prec == 0 else 2e-5
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


def test_matvec_general_parallel_base_matches_oracle(tsk):
    # a parallel base flow whose vorticity gradient is not proportional to U
    N = 48
    y = 2 * np.pi * np.arange(N) / N
    U = np.sin(y) + 0.5 * np.cos(2 * y)
    dO = np.sin(y) + 2.0 * np.cos(2 * y)          # -U''
    print("kolmo matvec general parallel base N=48", flush=True)
    op, ref = _op(tsk, N, base="parallel", U=U, dO=dO, alpha=0.75, Re=30.0)
    w = ref.project(W.kolmo_start_physical(N, 4))
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, w), x)
    yv = op.new_state()
    tsk.apply(op, x, yv)
    got = _to_phys(tsk, op, yv)
    want = ref.apply(w)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


@pytest.mark.parametrize("N", [32, 48])
def test_arnoldi_small_grid_same_steps_and_ritz_values(tsk, N):
    print(f"kolmo arnoldi N={N}", flush=True)
    op, ref = _op(tsk, N)
    w0 = W.kolmo_start_physical(N, 0)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, w0), x)
    r = tsk.arnoldi(op, 40, 6, 1e-8, v0=x)
    o = oracle_arnoldi(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), 40, 6, 1e-8,
                       T=ref.T)
    assert r["status"] == o["status"]
    assert r["n_matvec"] == o["n_matvec"]
    assert match_sets(r["lam"], o["lam"]) <= 1e-8


def test_arnoldi_full_config_fp64_matches_stored_oracle_run(tsk):
    print("kolmo arnoldi N=128 fp64 m=64 k=6 tol=1e-8", flush=True)
    c = W.KOLMO_128_FP64
    g = json.load(open(os.path.join(GOLD, "oracle_kolmo128_fp64.json")))
    N = c["N"]
    op, ref = _op(tsk, N)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, W.kolmo_start_physical(N, 0)), x)
    r = tsk.arnoldi(op, c["m"], c["k"], c["tol"], v0=x, want_vectors=True)
    assert r["status"] == 0
    # The leading eigenvalues are double (+-kx); their second copies only enter
    # the Krylov space through rounding, so late Hessenberg columns depend on
    # rounding order and the stop step may differ by a few matvecs.
    assert abs(r["n_matvec"] - g["n_matvec"]) <= 3
    assert np.all(r["res"] <= c["tol"])
    lam_o = np.array(g["lam_re"]) + 1j * np.array(g["lam_im"])
    assert match_sets(r["lam"], lam_o) <= 1e-8
    # and against the dense Galerkin eigenvalues of the operator (time error ~1e-9)
    blocks = galerkin_sinusoidal_blocks(N, c["alpha"], c["Re"])
    ev = np.concatenate([np.linalg.eigvals(A) for _, A in blocks.values()])
    assert match_sets(r["lam"], ev) <= 5e-8
    # Ritz vectors of the leading (multiplicity-2) pair: residual under the oracle
    X = r["X"].cpu().numpy()
    x0 = X[0]
    for part in (x0.real, x0.imag):
        if np.linalg.norm(part) < 1e-3:
            continue
        t = torch.from_numpy(part / np.linalg.norm(part)).cuda()
        ph = _to_phys(tsk, op, t)
        Mx = ref.apply(ph)
        rel = np.linalg.norm(Mx - r["mu"][0].real * ph) / np.linalg.norm(ph)
        assert rel <= 1e-7


def test_arnoldi_full_config_fp64_fixed_order_matches_oracle(tsk):
    # Same start vector, same number of steps (m = 53, tol = 0: no early stop),
    # as Algorithm 1 runs it: the six leading wanted Ritz values of H_53 agree
    # with the oracle's at the same order to 1e-8.
    print("kolmo arnoldi N=128 fp64 fixed order m=53", flush=True)
    c = W.KOLMO_128_FP64
    g = json.load(open(os.path.join(GOLD, "oracle_kolmo128_fp64_m53.json")))
    N = c["N"]
    op, _ = _op(tsk, N)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, W.kolmo_start_physical(N, 0)), x)
    r = tsk.arnoldi(op, 53, 12, 0.0, v0=x)
    assert r["status"] == g["status"] == 1
    assert r["n_matvec"] == g["n_matvec"] == 53
    lam_o = np.array(g["lam_re"]) + 1j * np.array(g["lam_im"])
    assert np.max(np.abs(r["lam"][:6] - lam_o[:6])) <= 1e-8
    # residual estimates of the same pairs agree to rounding of the late steps:
    # the sixth sits at the tolerance (oracle 9.3e-9), which decides the stop
    # step (53 on the oracle, 53-55 on the device)
    ro = np.array(g["res"][:6])
    big = ro >= 1e-10
    assert np.all(np.abs(np.log(r["res"][:6][big] / ro[big])) <= np.log(1.5))
    assert np.all(r["res"][:6] <= 2e-8)
    # every converged GPU value is a converged value of the oracle's H_53
    all_o = np.array(g["all_lam_re"]) + 1j * np.array(g["all_lam_im"])
    conv_o = all_o[np.array(g["all_res"]) <= 1e-8]
    for lam, res in zip(r["lam"], r["res"]):
        if res <= 1e-8:
            assert np.min(np.abs(conv_o - lam)) <= 1e-8


def test_seeded_start_matches_oracle_generator(tsk):
    from oracle.rng import normal
    N = 48
    print("kolmo seeded start N=48", flush=True)
    op, ref = _op(tsk, N)
    r = tsk.arnoldi(op, 30, 4, 1e-8, v0=None, seed=5)
    w0 = normal(N * N, 5).reshape(N, N)
    o = oracle_arnoldi(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), 30, 4, 1e-8,
                       T=ref.T)
    assert r["n_matvec"] == o["n_matvec"]
    assert match_sets(r["lam"], o["lam"]) <= 1e-8


def test_exact_eigenvector_start_breaks_down(tsk):
    N, Re = 48, 20.0
    print("kolmo breakdown", flush=True)
    op, ref = _op(tsk, N)
    x, y = ref.grid()
    w = np.repeat(np.cos(3 * y)[:, None], N, axis=1)
    s = op.new_state()
    tsk.from_physical(op, _phys(op, N, w), s)
    r = tsk.arnoldi(op, 10, 1, 1e-10, v0=s)
    assert r["status"] == 2 and r["n_matvec"] == 1
    assert abs(r["mu"][0] - np.exp(-9 * ref.T / Re)) < 1e-13


def test_invalid_sizes_and_parameters(tsk):
    for N in (100, 1024, 8):
        with pytest.raises(tsk.TskError) as e:
            tsk.create_kolmo2d(N, 0)
        assert e.value.status == tsk.TSK_EINVAL
    op = tsk.create_kolmo2d(32, 0)
    with pytest.raises(tsk.TskError):
        tsk.set_params_kolmo(op, 20.0, 0.5, 0.003, 1.0)
    with pytest.raises(tsk.TskError) as e:
        tsk.arnoldi(op, 10, 2, 1e-8)
    assert e.value.status == tsk.TSK_ESTATE


def test_hessenberg_columns_match_oracle_before_rounding_amplification(tsk):
    # Same start, fixed m: the first 20 columns of H agree elementwise.
    N, m = 128, 20
    print("kolmo N=128 H columns m=20", flush=True)
    op, ref = _op(tsk, N)
    w0 = W.kolmo_start_physical(N, 0)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, w0), x)
    r = tsk.arnoldi(op, m, 4, 0.0, v0=x)
    assert r["status"] == 1 and r["n_matvec"] == m
    H = tsk.last_hessenberg(op)
    o = oracle_arnoldi(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), m, 4, 0.0,
                       T=ref.T, keep_basis=False)
    assert np.max(np.abs(H - o["H"])) <= 1e-11


# Precision form: FP32 state, FFTs and IF-RK4; FP64 Gram-Schmidt sums, norms and
# Hessenberg QR.  Stated bound on |lambda_FP32 - lambda_oracle|: 2e-5 (about
# 100 FP32 unit roundoffs of the leading growth rates), measured ~5e-6.
FP32_LAMBDA_BOUND = 2e-5


@pytest.mark.parametrize("N,m", [(128, 64), (512, 96)])
def test_fp32_precision_form_within_stated_bound(tsk, N, m):
    print(f"kolmo fp32 N={N} m={m}", flush=True)
    g = json.load(open(os.path.join(GOLD, "oracle_kolmo128_fp64.json")))
    lam_o = np.array(g["lam_re"]) + 1j * np.array(g["lam_im"])
    op, _ = _op(tsk, N, prec=1)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, W.kolmo_start_physical(N, 0)), x)
    r = tsk.arnoldi(op, m, 6, 1e-8, v0=x)
    # six distinct eigenvalues (FP32 copies of the double ones are merged)
    assert r["n_ritz"] == 6
    lam = np.sort(r["lam"].real)[::-1]
    assert np.all(np.diff(lam) < -1e-3)
    assert match_sets(r["lam"], lam_o) <= FP32_LAMBDA_BOUND


@pytest.mark.parametrize("N,prec,base", [(128, 0, "kolmogorov"), (128, 1, "kolmogorov"), (128, 0, "general"),
                                         (48, 0, "general"), (256, 1, "kolmogorov"), (256, 0, "kolmogorov"),
                                         (96, 1, "general")])
def test_columns_per_wave_variants_agree_bitwise(tsk, N, prec, base):
    print(f"column-pair variant N={N} prec={prec} base={base}", flush=True)
    if base == "kolmogorov":
        op, _ = _op(tsk, N, prec=prec, T=0.05)
    else:
        y = 2 * np.pi * np.arange(N) / N
        op, _ = _op(tsk, N, prec=prec, T=0.05, base="parallel", U=np.sin(y) + 0.5 * np.cos(2 * y),
                    dO=np.sin(y) + 2.0 * np.cos(2 * y))
    x = op.new_state()
    tsk.from_physical(op, _phys(op, N, W.kolmo_start_physical(N, 9)), x)
    outs = []
    for c in (1, 2):
        tsk.set_tuning(op, c)
        assert tsk.get_tuning(op) == c
        y_ = op.new_state()
        tsk.apply(op, x, y_)
        outs.append(y_)
    assert torch.equal(outs[0], outs[1])
    tsk.set_tuning(op, 0)
    y_ = op.new_state()
    tsk.apply(op, x, y_)
    if base == "kolmogorov":
        # the default for the one-harmonic base is the spectral-coupling stepper:
        # the same operator, other rounding
        tol = 1e-13 if prec == 0 else 2e-6
        assert torch.max(torch.abs(y_ - outs[0])).item() <= tol * torch.max(torch.abs(outs[0])).item()
        assert not torch.equal(y_, outs[0])
        assert tsk.get_tuning(op) == -2
    else:
        assert torch.equal(y_, outs[0])       # autotuned: one of the two, same bits
        assert tsk.get_tuning(op) in (1, 2)
    with pytest.raises(tsk.TskError):
        tsk.set_tuning(op, 4)


@pytest.mark.parametrize("prec", [0, 1])
def test_bloch_stepper_512_matches_column_stepper(tsk, prec):
    # 512^2: Bloch sectors of 128 modes (two per lane, the cross-lane
    # 128-point transform) against the one-column-per-wave LDS stepper
    print(f"bloch 512 prec={prec}", flush=True)
    op, _ = _op(tsk, 512, prec=prec, T=0.05)
    x = op.new_state()
    tsk.from_physical(op, _phys(op, 512, W.kolmo_start_physical(512, 4)), x)
    tsk.set_tuning(op, 3)
    assert tsk.get_tuning(op) == -1
    yb = op.new_state()
    tsk.apply(op, x, yb)
    tsk.set_tuning(op, 1)
    assert tsk.get_tuning(op) == 1
    yc = op.new_state()
    tsk.apply(op, x, yc)
    tol = 1e-13 if prec == 0 else 2e-6
    assert torch.max(torch.abs(yb - yc)).item() <= tol * torch.max(torch.abs(yc)).item()
    assert torch.max(torch.abs(yc)).item() > 0
