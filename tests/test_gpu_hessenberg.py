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
