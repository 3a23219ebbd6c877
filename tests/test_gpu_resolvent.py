"""GPU parity of the resolvent by forced time integration (Sec. 2.3.2; Sec. 3.3.2)
against the CPU oracle, through the C ABI: the forced Crank-Nicolson response and
its adjoint, the gains of Lanczos on R^dagger R, and the paper's gain peak."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import golden
from oracle.cgle import CGLE
from oracle.resolvent import discrete_resolvent, forced_response

pytestmark = pytest.mark.gpu


def _pair(tsk, n, half_width, mu0, dt=0.01, T=1.0):
    ref = CGLE(n=n, half_width=half_width, mu0=mu0, dt=dt, T=T)
    op = tsk.create_cgle1d(n, half_width)
    tsk.set_params_cgle(op, 2.0, 0.2, -1.0, mu0, -0.01, dt, T)
    return op, ref


def _small(tsk):
    # short stable domain (least stable eigenvalue about -0.4): transients die fast
    return _pair(tsk, 48, 20.0, 0.0)


def _paper(tsk):
    # the paper's illustration: mu0 = 0.23, x in [-85, 85]; least stable
    # eigenvalue -0.151, so the transient is below 1e-15 after 230 time units
    return _pair(tsk, 400, 85.0, 0.23)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("omega", [-0.55, 0.3])
def test_forced_response_matches_oracle(tsk, omega):
    print(f"forced response n=48 omega={omega}", flush=True)
    op, ref = _small(tsk)
    tsk.set_resolvent(op, omega, 90.0)
    f, g = W.normal_complex(48, 1), W.normal_complex(48, 2)
    y = torch.zeros(48, dtype=torch.complex128, device="cuda")
    tsk.apply(op, _cuda(f), y)
    want = forced_response(ref, f, omega, 90.0)
    assert np.linalg.norm(y.cpu().numpy() - want) <= 1e-12 * np.linalg.norm(want)
    # and the closed form: the resolvent of L_h at the warped frequency
    closed = discrete_resolvent(ref, omega) @ f
    assert np.linalg.norm(y.cpu().numpy() - closed) <= 1e-10 * np.linalg.norm(closed)
    z = torch.zeros_like(y)
    tsk.apply_adjoint(op, _cuda(g), z)
    want_adj = forced_response(ref, g, omega, 90.0, adjoint=True)
    assert np.linalg.norm(z.cpu().numpy() - want_adj) <= 1e-12 * np.linalg.norm(want_adj)


def test_forced_response_at_the_paper_size(tsk):
    print("forced response n=400 omega=-0.55 t=230", flush=True)
    op, ref = _paper(tsk)
    tsk.set_resolvent(op, -0.55, 230.0)
    f = W.normal_complex(400, 3)
    y = torch.zeros(400, dtype=torch.complex128, device="cuda")
    tsk.apply(op, _cuda(f), y)
    want = forced_response(ref, f, -0.55, 230.0)
    assert np.linalg.norm(y.cpu().numpy() - want) <= 1e-10 * np.linalg.norm(want)
    closed = discrete_resolvent(ref, -0.55) @ f
    assert np.linalg.norm(y.cpu().numpy() - closed) <= 1e-9 * np.linalg.norm(closed)
    # <R f, g> = <f, R^H g>
    g = _cuda(W.normal_complex(400, 4))
    z = torch.zeros_like(y)
    tsk.apply_adjoint(op, g, z)
    lhs, rhs = torch.vdot(g, y).item(), torch.vdot(z, _cuda(f)).item()
    assert abs(lhs - rhs) <= 1e-10 * torch.linalg.norm(y).item() * torch.linalg.norm(g).item()


def test_lanczos_gains_match_the_dense_svd(tsk):
    print("resolvent gains n=48", flush=True)
    op, ref = _small(tsk)
    omega = -0.55
    tsk.set_resolvent(op, omega, 90.0)
    s = np.linalg.svd(discrete_resolvent(ref, omega), compute_uv=False)
    r = tsk.optimal_perturbation(op, 24, 3, 1e-9 * s[0] ** 2, v0=_cuda(W.normal_complex(48, 5)),
                                 want_vectors=True)
    assert r["status"] == 0
    assert np.max(np.abs(np.sort(r["gain"])[::-1] - s[:3] ** 2)) <= 1e-8 * s[0] ** 2
    # the optimal forcing: ||R f|| = sigma
    for sig, f in zip(r["sigma"], r["X"]):
        y = torch.zeros_like(f)
        tsk.apply(op, f.contiguous(), y)
        assert abs(torch.linalg.norm(y).item() - sig) <= 1e-8 * sig


def test_paper_gain_peak_and_disjoint_supports(tsk):
    # Sec. 2.3.2: gain close to 1000 near omega = -0.55; the optimal forcing
    # lies mostly in -20 <= x <= 0 and its response in 0 <= x <= 20
    g = golden("cgle_resolvent_peak.txt")
    op, ref = _paper(tsk)
    omegas = np.round(np.arange(-0.65, -0.449, 0.05), 2)
    gains = []
    for w in omegas:
        print(f"resolvent gain n=400 omega={w}", flush=True)
        tsk.set_resolvent(op, float(w), 230.0)
        s1 = np.linalg.svd(discrete_resolvent(ref, float(w)), compute_uv=False)[0]
        r = tsk.optimal_perturbation(op, 32, 1, 1e-7 * s1 ** 2, seed=1, want_vectors=True)
        assert r["status"] == 0
        assert abs(r["gain"][0] - s1 ** 2) <= 1e-7 * s1 ** 2
        gains.append(r["gain"][0])
    i = int(np.argmax(gains))
    assert abs(omegas[i] - g["omega_peak"]) <= g["omega_window"]
    assert g["gain_lower"] < gains[i] < g["gain_upper"]
    # supports at the peak: the forcing's energy centroid lies at x < 0, the
    # response's at x > 0
    tsk.set_resolvent(op, float(omegas[i]), 230.0)
    r = tsk.optimal_perturbation(op, 32, 1, 1e-7 * gains[i], seed=1, want_vectors=True)
    f = r["X"][0].contiguous()
    u = torch.zeros_like(f)
    tsk.apply(op, f, u)
    xf = np.sum(ref.x * np.abs(f.cpu().numpy()) ** 2) / np.sum(np.abs(f.cpu().numpy()) ** 2)
    xu = np.sum(ref.x * np.abs(u.cpu().numpy()) ** 2) / np.sum(np.abs(u.cpu().numpy()) ** 2)
    assert xf < 0.0 < xu


def test_resolvent_mode_validation_and_return_to_the_propagator(tsk):
    print("resolvent validation", flush=True)
    op, ref = _small(tsk)
    u = W.normal_complex(48, 6)
    y0 = torch.zeros(48, dtype=torch.complex128, device="cuda")
    tsk.apply(op, _cuda(u), y0)
    tsk.set_resolvent(op, -0.55, 10.0)
    with pytest.raises(tsk.TskError):
        tsk.set_resolvent(op, -0.55, -1.0)
    with pytest.raises(tsk.TskError):
        tsk.set_resolvent(op, float("nan"), 10.0)
    with pytest.raises(tsk.TskError):
        tsk.set_resolvent(op, -0.55, 0.001)   # below one time step
    tsk.set_resolvent(op, 0.0, 0.0)
    y1 = torch.zeros_like(y0)
    tsk.apply(op, _cuda(u), y1)
    assert torch.equal(y0, y1)
    assert np.linalg.norm(y1.cpu().numpy() - ref.apply(u)) <= 1e-12 * np.linalg.norm(y1.cpu().numpy())
    kop = tsk.create_kolmo2d(32, 0)
    tsk.set_params_kolmo(kop, 20.0, 0.5, 0.005, 1.0)
    tsk.set_base_kolmogorov(kop, 4)
    with pytest.raises(tsk.TskError):
        tsk.set_resolvent(kop, -0.55, 10.0)


def test_batched_frequency_sweep_matches_dense_and_single_runs(tsk):
    # one workgroup per frequency, all integrations of a pass in one launch
    print("batched resolvent sweep n=48, 8 frequencies", flush=True)
    omegas = np.linspace(-1.2, 0.2, 8)
    pairs = [_small(tsk) for _ in omegas]
    for (op, _), w in zip(pairs, omegas):
        tsk.set_resolvent(op, float(w), 90.0)
    ops = [p[0] for p in pairs]
    v0s = [_cuda(W.normal_complex(48, 20 + i)) for i in range(len(ops))]
    rb = tsk.batch_optimal_perturbation(ops, 24, 3, 1e-9, v0s=v0s, want_vectors=True)
    for i, ((op, ref), w) in enumerate(zip(pairs, omegas)):
        s = np.linalg.svd(discrete_resolvent(ref, float(w)), compute_uv=False)
        assert rb[i]["status"] == 0
        assert np.max(np.abs(rb[i]["gain"] - s[:3] ** 2)) <= 1e-8 * max(1.0, s[0] ** 2)
        r1 = tsk.optimal_perturbation(op, 24, 3, 1e-9, v0=v0s[i])
        assert r1["n_steps"] == rb[i]["n_steps"]
        assert np.max(np.abs(r1["gain"] - rb[i]["gain"])) <= 1e-12 * s[0] ** 2


def test_batched_paper_sweep_four_gains(tsk):
    # the paper's figure: the first four gains sigma_j^2 against omega
    print("batched resolvent sweep n=400, 6 frequencies, 4 gains", flush=True)
    omegas = np.linspace(-1.0, 0.0, 6)
    pairs = [_paper(tsk) for _ in omegas]
    for (op, _), w in zip(pairs, omegas):
        tsk.set_resolvent(op, float(w), 230.0)
    rb = tsk.batch_optimal_perturbation([p[0] for p in pairs], 48, 4, 1e-6, seeds=list(range(6)))
    for i, ((op, ref), w) in enumerate(zip(pairs, omegas)):
        s = np.linalg.svd(discrete_resolvent(ref, float(w)), compute_uv=False)
        assert rb[i]["status"] == 0
        assert np.max(np.abs(rb[i]["gain"] - s[:4] ** 2)) <= 1e-6 * s[0] ** 2 + 1e-6


def test_batched_propagators_and_mixed_sizes(tsk):
    # eigenvalue batches of Ginzburg-Landau propagators (one launch) and a batch of
    # two node counts (per-instance launches) give the single-run Ritz values
    print("batched cgle arnoldi", flush=True)
    ops = []
    for mu0, n in [(0.41, 256), (0.3, 256), (0.2, 256), (0.41, 200)]:
        op = tsk.create_cgle1d(n, 50.0)
        tsk.set_params_cgle(op, 2.0, 0.2, -1.0, mu0, -0.01, 0.01, 1.0)
        ops.append(op)
    for group in (ops[:3], [ops[0], ops[3]]):
        rb = tsk.batch_arnoldi(group, 64, 6, 1e-8, seeds=[0] * len(group))
        for op, r in zip(group, rb):
            r1 = tsk.arnoldi(op, 64, 6, 1e-8, seed=0)
            assert r["status"] == r1["status"] == 0 and r["n_matvec"] == r1["n_matvec"]
            assert np.max(np.abs(r["mu"] - r1["mu"])) <= 1e-12
