"""GPU parity of the Krylov-Schur path (Sec. 3.2.2) against the CPU oracle,
through the C ABI: the contraction kernel on its own (ordered real Schur form,
truncation, Arnoldi form) and whole restarted runs."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sl
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.kolmogorov import Kolmogorov, base_from_streamfunction, galerkin_sinusoidal_blocks
from oracle.krylov_schur import kept_count, krylov_schur as oracle_ks

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _fold(lam):
    # either member of a conjugate pair may fill the last wanted slot (equal |mu|)
    return np.array([complex(z.real, abs(z.imag)) for z in lam])


def _hessenberg(n, m, seed, scale=1.0):
    A = scale * (W.random_matrix(n, seed) / np.sqrt(n) + np.diag(np.linspace(-1, 2, n)))
    a = oracle_arnoldi(lambda v: A @ v, W.normal_real(n, seed + 1), m, m, 0.0)
    return np.ascontiguousarray(a["H"][:m, :m].real), float(a["beta"])


# (m, k, delta, p_max, scale): pair-split boundaries at m = 20, 64, 96; p = k
# forced by a small spectrum; p = p_max; every Ritz value wanted (delta = 5)
CASES = [(8, 2, 0.5, 0, 1.0), (20, 4, 0.1, 0, 1.0), (40, 6, 0.3, 12, 1.0), (64, 6, 0.1, 0, 1.0),
         (96, 10, 0.2, 40, 1.0), (30, 3, 5.0, 0, 1.0), (24, 5, 0.0, 0, 1.0), (16, 3, 0.0, 5, 1.0),
         (32, 4, 0.1, 0, 0.4), (3, 1, 0.1, 0, 1.0)]


@pytest.mark.parametrize("m,k,delta,pmax,scale", CASES)
def test_contraction_matches_ordered_schur_restart(tsk, m, k, delta, pmax, scale):
    print(f"ks contraction m={m} k={k} delta={delta} pmax={pmax} scale={scale}", flush=True)
    H, beta = _hessenberg(max(3 * m, 60), m, m, scale)
    pm = pmax or max(k, m // 2)
    mu_o, Y = np.linalg.eig(H)
    p, keep = kept_count(mu_o, k, m, delta, pm)
    kept = mu_o[keep]
    wanted = lambda re, im: int(np.argmin(np.abs(mu_o - (re + 1j * im)))) in set(keep)
    S, Q, sdim = sl.schur(H, output="real", sort=wanted)
    assert sdim == p
    mu, res, Hn, Wd, bnew = tsk.ks_contract(torch.from_numpy(H).cuda(), beta, k, delta, pmax)
    mu, res, Hn, Wm = mu.cpu().numpy(), res.cpu().numpy(), Hn.cpu().numpy(), Wd.cpu().numpy()
    assert Wm.shape == (m, p) and Hn.shape == (p + 1, p)
    nH = np.linalg.norm(H, 2)
    # Ritz values and residual estimates of H_m
    assert match_sets(mu, mu_o) <= 1e-10 * np.max(np.abs(mu_o))
    res_o = beta * np.abs(Y[-1]) / np.linalg.norm(Y, axis=0)
    for z, r in zip(mu, res):
        assert abs(r - res_o[int(np.argmin(np.abs(mu_o - z)))]) <= 1e-8 * beta
    # W: orthonormal basis of the kept invariant subspace of the ordered Schur form
    assert np.max(np.abs(Wm.T @ Wm - np.eye(p))) <= 1e-13
    assert np.max(sl.subspace_angles(Wm, Q[:, :p])) <= 1e-9
    # Arnoldi form: Hessenberg H_p = W^T H W, beta' = ||beta e_m^T Q_p|| at (p, p-1)
    Hp = Hn[:p]
    assert np.all(np.tril(Hp, -2) == 0.0)
    assert np.all(Hn[p, : p - 1] == 0.0) and Hn[p, p - 1] == bnew and bnew >= 0.0
    assert np.max(np.abs(Wm.T @ H @ Wm - Hp)) <= 1e-12 * nH
    assert np.max(np.abs(H @ Wm - Wm @ Hp)) <= 1e-11 * nH
    assert abs(bnew - np.linalg.norm(beta * Q[m - 1, :p])) <= 1e-12 * beta
    # e_m^T W = (beta' / beta) e_p^T: the relation M V_p = V_p H_p + beta' v_{m+1} e_p^T
    if p > 1:
        assert np.max(np.abs(Wm[m - 1, : p - 1])) <= 1e-13
    assert abs(Wm[m - 1, p - 1] - bnew / beta) <= 1e-13
    assert match_sets(np.linalg.eigvals(Hp), kept) <= 1e-9 * np.max(np.abs(kept))


def _general(tsk, N, seed, alpha=0.5, Re=20.0, dt=0.005, T=1.0, prec=0):
    U, V, Ox, Oy = base_from_streamfunction(W.random_base_modes(2, seed), N, alpha)
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    tsk.set_base_flow(op, U, V, Ox, Oy)
    return op, Kolmogorov(N, alpha, Re, dt, T, U, V, Ox, Oy)


def _kolmo(tsk, N, alpha=0.5, Re=20.0, dt=0.005, T=1.0, prec=0):
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    tsk.set_base_kolmogorov(op, 4)
    return op, Kolmogorov.kolmogorov(N, alpha, Re, dt, T, 4)


def _state(tsk, op, w):
    dt = torch.float64 if op.elem_bytes == 8 else torch.float32
    x = op.new_state()
    tsk.from_physical(op, torch.from_numpy(np.ascontiguousarray(w)).to(dt).cuda().reshape(-1), x)
    return x


@pytest.mark.parametrize("m", [16, 20])
def test_general_base_run_matches_oracle_restart_by_restart(tsk, m):
    # no symmetry: simple eigenvalues, so the contraction sizes are robust to rounding
    N = 32
    print(f"ks general base N={N} m={m}", flush=True)
    op, ref = _general(tsk, N, seed=100 + N)
    w0 = W.kolmo_start_physical(N, 7)
    r = tsk.krylov_schur(op, m, 6, 1e-8, delta=0.1, v0=_state(tsk, op, w0))
    o = oracle_ks(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), m, 6, 1e-8, delta=0.1,
                  T=ref.T)
    assert r["status"] == o["status"] == 0
    assert r["n_restarts"] == o["n_restarts"] and r["n_matvec"] == o["n_matvec"]
    assert r["kept_last"] == o["p_hist"][-1]
    assert np.all(r["res"] <= 1e-8)
    assert match_sets(_fold(r["lam"]), _fold(o["lam"])) <= 1e-8


def _distinct(lam, tol=1e-7):
    out = []
    for z in sorted(lam, key=lambda z: -z.real):
        if all(abs(z - w) > tol for w in out):
            out.append(z)
    return np.array(out)


def test_kolmogorov_run_matches_oracle(tsk):
    # The x-translation symmetry makes every real eigenvalue with kx != 0 double.
    # Its second copy enters the Krylov space only through rounding, and
    # restarts amplify it, so a run may resolve both copies (two of the k slots)
    # or one: compare the distinct leading values, and check every value
    # against the dense Galerkin spectrum.
    N, m, k = 32, 24, 6
    print(f"ks kolmogorov N={N} m={m}", flush=True)
    op, ref = _kolmo(tsk, N)
    w0 = W.kolmo_start_physical(N, 0)
    r = tsk.krylov_schur(op, m, k, 1e-8, delta=0.1, v0=_state(tsk, op, w0))
    o = oracle_ks(lambda v: ref.apply(v.reshape(N, N)).ravel(), ref.project(w0).ravel(), m, k, 1e-8, delta=0.1,
                  T=ref.T)
    assert r["status"] == o["status"] == 0
    assert abs(r["n_matvec"] - o["n_matvec"]) <= m
    dg, do = _distinct(r["lam"]), _distinct(o["lam"])
    n = min(len(dg), len(do))
    assert n >= k // 2
    assert np.max(np.abs(dg[:n] - do[:n])) <= 1e-8
    blocks = galerkin_sinusoidal_blocks(N, 0.5, 20.0)
    ev = np.concatenate([np.linalg.eigvals(A) for _, A in blocks.values()])
    for lam in r["lam"]:
        assert np.min(np.abs(ev - lam)) <= 5e-8


def test_without_contraction_equals_arnoldi_at_order_m(tsk):
    N, m, k = 32, 24, 6
    print("ks no restart N=32 m=24", flush=True)
    op, ref = _general(tsk, N, seed=5)
    x = _state(tsk, op, W.kolmo_start_physical(N, 1))
    r = tsk.krylov_schur(op, m, k, 0.0, max_restarts=0, v0=x)
    a = tsk.arnoldi(op, m, k, 0.0, v0=x)
    assert r["status"] == a["status"] == 1
    assert r["n_matvec"] == a["n_matvec"] == m and r["n_restarts"] == 0
    assert match_sets(_fold(r["lam"]), _fold(a["lam"])) <= 1e-12
    assert np.max(np.abs(np.sort(r["res"]) - np.sort(a["res"]))) <= 1e-12


def test_ritz_vectors_are_eigenvectors_of_the_oracle_operator(tsk):
    N, m, k = 32, 16, 4
    print("ks ritz vectors N=32", flush=True)
    op, ref = _general(tsk, N, seed=132)
    r = tsk.krylov_schur(op, m, k, 1e-9, delta=0.1, seed=3, want_vectors=True)
    assert r["status"] == 0 and r["n_restarts"] >= 1
    X = r["X"].cpu().numpy()
    for mu, x in zip(r["mu"], X):
        # physical fields of Re and Im parts; M x = mu x for the complex vector
        phys = []
        for part in (x.real, x.imag):
            out = torch.zeros(N * N, dtype=torch.float64, device="cuda")
            tsk.to_physical(op, torch.from_numpy(np.ascontiguousarray(part)).cuda(), out)
            phys.append(out.cpu().numpy().reshape(N, N))
        z = phys[0] + 1j * phys[1]
        Mz = ref.apply(phys[0]) + 1j * ref.apply(phys[1])
        assert np.linalg.norm(Mz - mu * z) <= 1e-7 * np.linalg.norm(z)


def test_full_config_restarted_matches_stored_oracle_arnoldi(tsk):
    c = W.KOLMO_128_FP64
    N = c["N"]
    print("ks kolmogorov N=128 fp64 m=32 k=6", flush=True)
    g = json.load(open(os.path.join(GOLD, "oracle_kolmo128_fp64.json")))
    op, ref = _kolmo(tsk, N)
    x = _state(tsk, op, W.kolmo_start_physical(N, 0))
    r = tsk.krylov_schur(op, 32, c["k"], c["tol"], delta=0.1, v0=x)
    assert r["status"] == 0 and r["n_restarts"] >= 1
    assert np.all(r["res"] <= c["tol"])
    lam_o = np.array(g["lam_re"]) + 1j * np.array(g["lam_im"])
    # every converged value is one of the oracle's leading eigenvalues
    for lam in r["lam"]:
        assert np.min(np.abs(lam_o - lam)) <= 1e-8


def test_fp32_run_within_stated_bound(tsk):
    N, m, k = 64, 24, 6
    print("ks fp32 N=64", flush=True)
    op64, _ = _general(tsk, N, seed=9)
    op32, _ = _general(tsk, N, seed=9, prec=1)
    w0 = W.kolmo_start_physical(N, 2)
    r64 = tsk.krylov_schur(op64, m, k, 1e-8, v0=_state(tsk, op64, w0))
    r32 = tsk.krylov_schur(op32, m, k, 1e-8, v0=_state(tsk, op32, w0))
    assert r64["status"] == 0 and r32["status"] == 0
    mu64 = _fold(r64["mu"])
    for mu in _fold(r32["mu"]):
        assert np.min(np.abs(mu64 - mu)) <= 2e-5 * abs(mu)


def test_exact_eigenvector_start_breaks_down(tsk):
    N, Re = 32, 20.0
    print("ks breakdown", flush=True)
    op, ref = _kolmo(tsk, N)
    x, y = ref.grid()
    w = np.repeat(np.cos(3 * y)[:, None], N, axis=1)
    r = tsk.krylov_schur(op, 10, 1, 1e-10, v0=_state(tsk, op, w))
    assert r["status"] == 2 and r["n_matvec"] == 1 and r["n_restarts"] == 0
    assert abs(r["mu"][0] - np.exp(-9 * ref.T / Re)) < 1e-13


def test_validation(tsk):
    print("ks validation", flush=True)
    op, _ = _kolmo(tsk, 32)
    for args in [dict(m=7, k=6), dict(m=97, k=6), dict(m=20, k=0)]:
        with pytest.raises(tsk.TskError):
            tsk.krylov_schur(op, args["m"], args["k"], 1e-8)
    with pytest.raises(tsk.TskError):
        tsk.krylov_schur(op, 20, 6, 1e-8, p_max=19)
    with pytest.raises(tsk.TskError):
        tsk.krylov_schur(op, 20, 6, 1e-8, p_max=5)
    with pytest.raises(tsk.TskError):
        tsk.krylov_schur(op, 20, 6, 1e-8, delta=-0.1)
    cg = tsk.create_cgle1d(256)
    tsk.set_params_cgle(cg, 2.0, 0.2, -1.0, 0.41, -0.01, 0.01, 1.0)
    with pytest.raises(tsk.TskError) as e:
        tsk.krylov_schur(cg, 20, 6, 1e-8)
    assert "real" in str(e.value)
    H = torch.eye(4, dtype=torch.float64, device="cuda")
    with pytest.raises(tsk.TskError):
        tsk.ks_contract(H, 1.0, 3)  # m < k + 2
    H = torch.full((6, 6), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(tsk.TskError):
        tsk.ks_contract(H, 1.0, 2)
