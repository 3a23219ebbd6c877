"""Device Hessenberg eigensolver (tsk_hessenberg_ritz) against LAPACK."""
import numpy as np
import pytest
import torch

import workloads as W
from conftest import match_sets

pytestmark = pytest.mark.gpu


def _hess(p, seed, cplx, scale=None):
    A = W.random_matrix(p, seed, complex_=cplx)
    H = np.triu(A, -1)
    if scale is not None:  # graded matrix
        d = scale ** np.arange(p)
        H = H * d[:, None] / d[None, :]
    return H


@pytest.mark.parametrize("p", [1, 2, 3, 7, 40, 64, 96])
@pytest.mark.parametrize("cplx", [False, True])
def test_eigenpairs_match_lapack(tsk, p, cplx):
    print(f"hessenberg p={p} complex={cplx}", flush=True)
    H = _hess(p, 10 + p, cplx)
    beta = 0.37
    mu, Y, res = tsk.hessenberg_ritz(torch.from_numpy(H.astype(complex)).cuda(), beta)
    mu, Y, res = mu.cpu().numpy(), Y.cpu().numpy(), res.cpu().numpy()
    ev = np.linalg.eigvals(H)
    nrm = np.linalg.norm(H, 2)
    assert match_sets(mu, ev) <= 1e-9 * nrm
    for i in range(p):
        y = Y[:, i]
        assert abs(np.linalg.norm(y) - 1) < 1e-12
        assert np.linalg.norm(H @ y - mu[i] * y) <= 1e-11 * nrm
        assert abs(res[i] - beta * abs(y[-1])) <= 1e-15 + 1e-13 * res[i]


def test_graded_and_structured_matrices(tsk):
    # graded entries, a Jordan-like near-defective block, exact conjugate pairs
    cases = [_hess(30, 3, False, scale=0.5), np.diag(np.full(12, 0.5)) + np.diag(np.full(11, 1.0), -1) * 1e-3]
    rot = np.zeros((10, 10))
    for i in range(0, 10, 2):
        a, b = 0.9 - 0.05 * i, 0.3 + 0.02 * i
        rot[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
    Q, _ = np.linalg.qr(W.normal_real((10, 10), 4))
    from scipy.linalg import hessenberg
    cases.append(hessenberg(Q @ rot @ Q.T))
    for H in cases:
        print(f"structured p={H.shape[0]}", flush=True)
        mu, Y, res = tsk.hessenberg_ritz(torch.from_numpy(H.astype(complex)).cuda(), 1.0)
        mu = mu.cpu().numpy()
        ev = np.linalg.eigvals(H)
        assert match_sets(mu, ev) <= 1e-7 * max(1.0, np.linalg.norm(H, 2))


# ---- the real double-shift solver (real operators) -------------------------------------
def _real_check(tsk, H, beta, tol_ev=1e-9, check_res=True):
    mu, res = tsk.hessenberg_ritz_real(torch.from_numpy(H).cuda(), beta)
    mu, res = mu.cpu().numpy(), res.cpu().numpy()
    ev, V = np.linalg.eig(H)
    nrm = max(1.0, np.linalg.norm(H, 2))
    assert match_sets(mu, ev) <= tol_ev * nrm
    # conjugate pairs come as (a + ib, a - ib) in consecutive entries
    for i in range(len(mu)):
        if mu[i].imag > 0:
            assert abs(mu[i + 1] - np.conj(mu[i])) <= 1e-14 * nrm
    if check_res:
        V = V / np.linalg.norm(V, axis=0, keepdims=True)
        for i in range(len(mu)):
            j = int(np.argmin(np.abs(ev - mu[i])))
            assert abs(res[i] - beta * abs(V[-1, j])) <= 1e-9 * max(beta, 1e-300) + 1e-8 * res[i], (i, res[i])
    return mu, res


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 40, 64, 96])
def test_real_solver_matches_lapack(tsk, p):
    print(f"real hessenberg p={p}", flush=True)
    _real_check(tsk, _hess(p, 20 + p, False), 0.61)


def test_real_solver_structured_matrices(tsk):
    from scipy.linalg import hessenberg
    # graded
    _real_check(tsk, _hess(30, 5, False, scale=0.5), 1.0, tol_ev=1e-7, check_res=False)
    # rotation blocks: exact complex pairs of known values
    rot = np.zeros((12, 12))
    for i in range(0, 12, 2):
        a, b = 0.9 - 0.05 * i, 0.3 + 0.02 * i
        rot[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
    Q, _ = np.linalg.qr(W.normal_real((12, 12), 6))
    mu, _ = _real_check(tsk, hessenberg(Q @ rot @ Q.T), 1.0, tol_ev=1e-10, check_res=False)
    # a 2x2 block with real eigenvalues next to a pair, already deflated from the rest
    H = np.zeros((6, 6))
    H[:2, :2] = [[1.0, 2.0], [3.0, 4.0]]
    H[2:4, 2:4] = [[0.5, -1.0], [2.0, 0.5]]
    H[4:, 4:] = [[-1.0, 0.25], [1.0, -1.0]]
    H[np.triu_indices(6, 2)] = 0.1
    _real_check(tsk, H, 0.3)
    # near-defective: a small-coupling chain of equal diagonal entries
    D = np.diag(np.full(12, 0.5)) + np.diag(np.full(11, 1.0), -1) * 1e-3
    _real_check(tsk, D, 1.0, tol_ev=1e-7, check_res=False)


def test_real_solver_rejects_non_finite_input(tsk):
    H = _hess(8, 3, False)
    H[2, 3] = np.nan
    with pytest.raises(tsk.TskError) as e:
        tsk.hessenberg_ritz_real(torch.from_numpy(H).cuda(), 1.0)
    assert e.value.status == tsk.TSK_ENONFINITE
