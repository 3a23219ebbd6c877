"""The non-allocating eigensolver entry point (tsk_hessenberg_ritz_real_noalloc)
against the allocating one (tsk_hessenberg_ritz_real), through the C ABI: the
same kernel on the same input, so the outputs agree bit for bit; two calls in
a row, the second smaller, so what the first left in the shared scratch must
not leak into the second."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _hessenberg(p, ldh, seed):
    """A real upper Hessenberg p x p matrix, column-major with leading dimension
    ldh (rows p..ldh-1 of each column hold junk the solver must not read)."""
    A = np.triu(W.normal_real((p, p), seed), -1)
    buf = np.full((p, ldh), 7.5)          # column j = buf[j]
    buf[:, :p] = A.T
    return A, torch.from_numpy(buf.ravel().copy()).cuda()


def _alloc_version(tsk, Hbuf, ldh, p, beta):
    mu = torch.zeros(p, dtype=torch.complex128, device="cuda")
    res = torch.zeros(p, dtype=torch.float64, device="cuda")
    st = tsk.load().tsk_hessenberg_ritz_real(C.c_void_p(Hbuf.data_ptr()), ldh, p, beta, C.c_void_p(mu.data_ptr()),
                                              C.c_void_p(res.data_ptr()), tsk._stream())
    assert st == 0, tsk.load().tsk_last_error()
    return mu, res


def _noalloc_version(tsk, Hbuf, ldh, p, beta):
    mu = torch.full((p,), 3.0 + 3.0j, dtype=torch.complex128, device="cuda")
    res = torch.full((p,), 9.0, dtype=torch.float64, device="cuda")
    tsk.hessenberg_ritz_real_noalloc(Hbuf, ldh, p, beta, mu, res)
    return mu, res


def test_noalloc_eigensolver_matches_allocating_one_twice(tsk):
    torch.cuda.set_device(0)
    for p, ldh, seed, beta in ((90, 97, 11, 0.37), (23, 40, 12, 1.5)):
        print(f"noalloc eigensolver p={p} ldh={ldh}", flush=True)
        A, Hbuf = _hessenberg(p, ldh, seed)
        mu_a, res_a = _alloc_version(tsk, Hbuf, ldh, p, beta)
        mu_n, res_n = _noalloc_version(tsk, Hbuf, ldh, p, beta)
        torch.cuda.synchronize()
        assert torch.equal(mu_a, mu_n)
        assert torch.equal(res_a, res_n)
        # and the eigenvalues are those of A (LAPACK), as for the allocating solver
        ev = np.linalg.eigvals(A)
        got = mu_n.cpu().numpy()
        for z in ev:
            assert np.min(np.abs(got - z)) <= 1e-9 * np.linalg.norm(A)


def test_noalloc_rejects_sizes_beyond_its_scratch(tsk):
    lib = tsk.load()
    H = torch.zeros(98 * 97, dtype=torch.float64, device="cuda")
    mu = torch.zeros(97, dtype=torch.complex128, device="cuda")
    res = torch.zeros(97, dtype=torch.float64, device="cuda")
    args = (C.c_void_p(mu.data_ptr()), C.c_void_p(res.data_ptr()), tsk._stream())
    assert lib.tsk_hessenberg_ritz_real_noalloc(C.c_void_p(H.data_ptr()), 97, 97, 1.0, *args) == tsk.TSK_EINVAL
    assert b"96" in lib.tsk_last_error()
    assert lib.tsk_hessenberg_ritz_real_noalloc(C.c_void_p(H.data_ptr()), 98, 50, 1.0, *args) == tsk.TSK_EINVAL
    assert b"97" in lib.tsk_last_error()
    assert lib.tsk_hessenberg_ritz_real_noalloc(C.c_void_p(H.data_ptr()), 10, 20, 1.0, *args) == tsk.TSK_EINVAL
    assert lib.tsk_hessenberg_ritz_real_noalloc(None, 20, 20, 1.0, *args) == tsk.TSK_EINVAL
    # a valid call still works after the rejected ones
    A, Hbuf = _hessenberg(8, 8, 3)
    mu8, res8 = _noalloc_version(tsk, Hbuf, 8, 8, 0.5)
    ma, ra = _alloc_version(tsk, Hbuf, 8, 8, 0.5)
    assert torch.equal(mu8, ma) and torch.equal(res8, ra)
