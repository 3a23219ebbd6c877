"""GPU parity of the Ginzburg-Landau path (Crank-Nicolson matvec + Arnoldi-CGS2 +
device Hessenberg QR) against the CPU oracle, through the C ABI."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets
from oracle.arnoldi import arnoldi as oracle_arnoldi
from oracle.cgle import CGLE

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _op(tsk, n=256, **kw):
    c = dict(W.CGLE)
    c.update(kw)
    op = tsk.create_cgle1d(n, c["half_width"])
    tsk.set_params_cgle(op, c["U"], c["c_u"], c["c_d"], c["mu0"], c["mu2"], c["dt"], c["T"])
    ref = CGLE(n=n, half_width=c["half_width"], U=c["U"], c_u=c["c_u"], c_d=c["c_d"], mu0=c["mu0"],
               mu2=c["mu2"], dt=c["dt"], T=c["T"])
    return op, ref


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [256, 100, 1024, 2])
def test_matvec_matches_oracle(tsk, n):
    print(f"cgle matvec n={n}", flush=True)
    op, ref = _op(tsk, n)
    u = W.cgle_start(n, 5)
    x = _dev(u)
    y = op.new_state()
    tsk.apply(op, x, y)
    got = y.cpu().numpy()
    want = ref.apply(u)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)




def test_arnoldi_full_config_parity(tsk):
    print("cgle arnoldi n=256 m=64 k=6 tol=1e-8", flush=True)
    c = W.CGLE
    g = json.load(open(os.path.join(GOLD, "oracle_cgle256.json")))
    op, ref = _op(tsk)
    v0 = _dev(W.cgle_start(256, 0))
    r = tsk.arnoldi(op, c["m"], c["k"], c["tol"], v0=v0, want_vectors=True)
    assert r["status"] == 0
    assert r["n_matvec"] == g["n_matvec"]
    lam_o = np.array(g["lam_re"]) + 1j * np.array(g["lam_im"])
    assert match_sets(r["lam"], lam_o) <= 1e-8
    assert np.all(r["res"] <= c["tol"])
    # Ritz vectors: unit norm, and their true residual under the oracle operator
    # is at the level of the reported estimate
    X = r["X"].cpu().numpy()
    for x, mu, res in zip(X, r["mu"], r["res"]):
        assert abs(np.linalg.norm(x) - 1) < 1e-10
        true = np.linalg.norm(ref.apply(x) - mu * x)
        assert true <= 10 * res + 1e-11


def test_hessenberg_and_basis_match_oracle_at_fixed_m(tsk):
    print("cgle arnoldi fixed m=20 (tol=0)", flush=True)
    op, ref = _op(tsk)
    u0 = W.cgle_start(256, 1)
    r = tsk.arnoldi(op, 20, 4, 0.0, v0=_dev(u0))
    assert r["status"] == 1 and r["n_matvec"] == 20
    H = tsk.last_hessenberg(op)
    o = oracle_arnoldi(ref.apply, u0, 20, 4, 0.0, T=ref.T)
    assert np.max(np.abs(H - o["H"])) <= 1e-10
    assert match_sets(r["mu"], o["mu"]) <= 1e-10


def test_seeded_start_matches_oracle_generator(tsk):
    from oracle.rng import normal
    print("cgle arnoldi seeded start", flush=True)
    op, ref = _op(tsk)
    r = tsk.arnoldi(op, 30, 3, 1e-8, v0=None, seed=11)
    z = normal(512, 11)
    u0 = z[0::2] + 1j * z[1::2]
    o = oracle_arnoldi(ref.apply, u0, 30, 3, 1e-8, T=ref.T)
    assert r["n_matvec"] == o["n_matvec"]
    assert match_sets(r["lam"], o["lam"]) <= 1e-8


def test_eigenvector_start_stops_after_one_matvec(tsk):
    # a LAPACK eigenvector of L_h is an eigenvector of the discrete propagator to
    # rounding: the first Ritz pair is exact (converged, or a happy breakdown)
    print("cgle eigenvector start", flush=True)
    op, ref = _op(tsk)
    lam, vec = np.linalg.eig(ref.matrix())
    i = int(np.argmax(lam.real))
    r = tsk.arnoldi(op, 10, 1, 1e-8, v0=_dev(vec[:, i].copy()))
    assert r["status"] in (0, 2) and r["n_matvec"] == 1
    z = ref.dt * lam[i]
    mu = ((1 + z / 2) / (1 - z / 2)) ** ref.nsteps
    assert abs(r["mu"][0] - mu) <= 1e-12


def test_invalid_arguments_are_rejected(tsk):
    op, _ = _op(tsk)
    v0 = _dev(W.cgle_start(256, 0))
    for m, k in ((97, 6), (4, 6), (5, 0)):
        with pytest.raises(tsk.TskError) as e:
            tsk.arnoldi(op, m, k, 1e-8, v0=v0)
        assert e.value.status == tsk.TSK_EINVAL
    bad = v0.clone()
    bad[3] = float("nan")
    with pytest.raises(tsk.TskError) as e:
        tsk.arnoldi(op, 10, 2, 1e-8, v0=bad)
    assert e.value.status == tsk.TSK_ENONFINITE
    with pytest.raises(tsk.TskError) as e:
        tsk.arnoldi(op, 10, 2, 1e-8, v0=torch.zeros_like(v0))
    assert e.value.status == tsk.TSK_EINVAL
    with pytest.raises(tsk.TskError) as e:
        tsk.set_params_cgle(op, 2.0, 0.2, -1.0, 0.41, -0.01, 0.01, 1.005)
    assert e.value.status == tsk.TSK_EINVAL
    fresh = tsk.create_cgle1d(64, 50.0)
    with pytest.raises(tsk.TskError) as e:
        tsk.apply(fresh, fresh.new_state(), fresh.new_state())
    assert e.value.status == tsk.TSK_ESTATE
