"""Thin ctypes binding of libtsk (include/tsk.h).  Argument marshalling only:
every step of the computation runs in the HIP library.  PyTorch supplies device
memory (tensors as buffers) and the current HIP stream.

The binding refuses to work without the built library: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsk.so")

TSK_OK, TSK_NOT_CONVERGED, TSK_BREAKDOWN = 0, 1, 2
TSK_EINVAL, TSK_ENOMEM, TSK_EHIP, TSK_ENONFINITE, TSK_ESTATE, TSK_EEIG = -1, -2, -3, -4, -5, -6
TSK_FP64, TSK_FP32 = 0, 1


class TskError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class FpInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("time_steps", C.c_int64), ("basis_dim", C.c_int),
                ("residual", C.c_double), ("ms_total", C.c_double)]


class KsInfo(C.Structure):
    _fields_ = [("n_matvec", C.c_int), ("n_restarts", C.c_int), ("n_ritz", C.c_int),
                ("n_converged", C.c_int), ("status", C.c_int), ("kept_last", C.c_int),
                ("beta", C.c_double), ("ms_total", C.c_double), ("ms_apply", C.c_double)]


class ArnoldiInfo(C.Structure):
    _fields_ = [("n_matvec", C.c_int), ("n_ritz", C.c_int), ("n_converged", C.c_int),
                ("status", C.c_int), ("beta", C.c_double), ("ms_total", C.c_double),
                ("ms_apply", C.c_double)]


_lib = None


def load():
    """Load libtsk.so (built by paper_1804_03859_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtsk.so not found at {LIB_PATH}: build it with "
                          "`python -m paper_1804_03859_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, u64 = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_uint64
    P = C.POINTER
    sig = {
        "tsk_create_cgle1d": [P(vp), i32, f64, vp],
        "tsk_set_params_cgle": [vp, f64, f64, f64, f64, f64, f64, f64],
        "tsk_create_kolmo2d": [P(vp), i32, i32, vp],
        "tsk_set_params_kolmo": [vp, f64, f64, f64, f64],
        "tsk_set_base_parallel": [vp, P(f64), P(f64)],
        "tsk_set_base_kolmogorov": [vp, i32],
        "tsk_set_base_flow": [vp, P(f64), P(f64), P(f64), P(f64)],
        "tsk_state_dim": [vp, P(i64), P(i32), P(i32)],
        "tsk_set_tuning": [vp, i32],
        "tsk_get_tuning": [vp, P(i32)],
        "tsk_set_stop_rule": [vp, f64, f64],
        "tsk_set_stepper_waves": [vp, i32],
        "tsk_get_stepper_waves": [vp, P(i32)],
        "tsk_from_physical": [vp, vp, vp],
        "tsk_to_physical": [vp, vp, vp],
        "tsk_apply": [vp, vp, vp],
        "tsk_arnoldi": [vp, i32, i32, f64, vp, u64, P(f64), P(f64), P(f64), vp, P(ArnoldiInfo)],
        "tsk_batch_arnoldi": [P(vp), i32, i32, i32, f64, P(vp), P(u64), P(f64), P(f64), P(f64), P(vp),
                              P(ArnoldiInfo)],
        "tsk_apply_adjoint": [vp, vp, vp],
        "tsk_set_resolvent": [vp, f64, f64],
        "tsk_batch_optimal_perturbation": [P(vp), i32, i32, i32, f64, P(vp), P(u64), P(f64), P(f64), P(vp),
                                           P(ArnoldiInfo)],
        "tsk_set_nonlinear": [vp, i32, f64, P(f64)],
        "tsk_laminar_state": [vp, vp],
        "tsk_nonlinear_step": [vp, vp, vp, i32],
        "tsk_set_base_from_state": [vp, vp],
        "tsk_sfd": [vp, vp, f64, f64, i32, f64, i32, P(f64), P(FpInfo)],
        "tsk_rpm": [vp, vp, i32, i32, f64, f64, i32, P(f64), P(FpInfo)],
        "tsk_boostconv": [vp, vp, i32, f64, i32, P(f64), P(FpInfo)],
        "tsk_optimal_perturbation": [vp, i32, i32, f64, vp, u64, P(f64), P(f64), vp, P(ArnoldiInfo)],
        "tsk_krylov_schur": [vp, i32, i32, f64, f64, i32, i32, vp, u64, P(f64), P(f64), P(f64), vp, P(KsInfo)],
        "tsk_batch_krylov_schur": [P(vp), i32, i32, i32, f64, f64, i32, i32, P(vp), P(u64), P(f64), P(f64), P(f64),
                                   P(vp), P(KsInfo)],
        "tsk_ks_contract": [vp, i32, i32, f64, i32, f64, i32, vp, vp, vp, vp, P(i32), P(f64), vp],
        "tsk_last_hessenberg": [vp, P(f64), P(i32), P(i32)],
        "tsk_last_basis": [vp, P(vp), P(i64)],
        "tsk_hessenberg_ritz": [vp, i32, i32, f64, vp, vp, vp, vp],
        "tsk_hessenberg_ritz_real": [vp, i32, i32, f64, vp, vp, vp],
        "tsk_hessenberg_ritz_real_noalloc": [vp, i32, i32, f64, vp, vp, vp],
        "tsk_normal_fill": [vp, i64, u64, vp],
        "tsk_mlp_create": [P(vp), i32, P(f64), P(f64), vp],
        "tsk_mlp_param_count": [vp, P(i64)],
        "tsk_mlp_init": [vp, u64],
        "tsk_mlp_set_params": [vp, vp],
        "tsk_mlp_get_params": [vp, vp],
        "tsk_mlp_forward": [vp, vp, i32, vp],
        "tsk_mlp_gradients": [vp, vp, vp, i32, vp, P(f64)],
        "tsk_mlp_train": [vp, vp, vp, i32, i32, f64, P(f64)],
        "tsk_ritz_block_target": [vp, vp, i32, P(i32), vp],
        "tsk_mlp_start": [vp, vp, f64, f64, f64, u64, vp, P(i32)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.tsk_destroy.argtypes = [vp]
    lib.tsk_destroy.restype = None
    lib.tsk_mlp_destroy.argtypes = [vp]
    lib.tsk_mlp_destroy.restype = None
    lib.tsk_status_str.argtypes = [C.c_int]
    lib.tsk_status_str.restype = C.c_char_p
    lib.tsk_last_error.argtypes = []
    lib.tsk_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def exported_symbols():
    """Names the binding expects the library to export (all of include/tsk.h)."""
    return ["tsk_create_cgle1d", "tsk_set_params_cgle", "tsk_create_kolmo2d", "tsk_set_params_kolmo",
            "tsk_set_base_parallel", "tsk_set_base_kolmogorov", "tsk_set_base_flow", "tsk_set_tuning",
            "tsk_get_tuning", "tsk_set_stop_rule", "tsk_set_stepper_waves", "tsk_get_stepper_waves",
            "tsk_state_dim",
            "tsk_from_physical", "tsk_to_physical", "tsk_apply", "tsk_arnoldi", "tsk_batch_arnoldi",
            "tsk_krylov_schur", "tsk_batch_krylov_schur", "tsk_ks_contract", "tsk_apply_adjoint", "tsk_optimal_perturbation",
            "tsk_set_resolvent", "tsk_batch_optimal_perturbation",
            "tsk_set_nonlinear", "tsk_laminar_state", "tsk_nonlinear_step", "tsk_set_base_from_state", "tsk_sfd",
            "tsk_rpm", "tsk_boostconv",
            "tsk_last_hessenberg",
            "tsk_last_basis", "tsk_hessenberg_ritz", "tsk_hessenberg_ritz_real",
            "tsk_hessenberg_ritz_real_noalloc", "tsk_normal_fill", "tsk_destroy", "tsk_status_str",
            "tsk_last_error", "tsk_mlp_create", "tsk_mlp_param_count", "tsk_mlp_init", "tsk_mlp_set_params",
            "tsk_mlp_get_params", "tsk_mlp_forward", "tsk_mlp_gradients", "tsk_mlp_train",
            "tsk_ritz_block_target", "tsk_mlp_start", "tsk_mlp_destroy"]


def _check(st, allow_positive=True):
    if st < 0 or (st > 0 and not allow_positive):
        lib = load()
        raise TskError(st, lib.tsk_last_error().decode())
    return st


def _stream(stream=None):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _need(t, numel, dtype, what):
    """Host-side check that a device buffer has the size and type the kernels
    assume (the library itself only sees raw pointers)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA/HIP tensor")
    if t.dtype != dtype or t.numel() != numel or not t.is_contiguous():
        raise ValueError(f"{what}: expected {numel} contiguous {dtype}, got {tuple(t.shape)} {t.dtype}")


def _dbl(arr):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


class Op:
    """Owning wrapper of a tsk_op handle."""

    def __init__(self, handle, kind):
        self.h = handle
        self.kind = kind
        n, c, b = C.c_int64(), C.c_int(), C.c_int()
        _check(load().tsk_state_dim(self.h, C.byref(n), C.byref(c), C.byref(b)))
        self.n, self.is_complex, self.elem_bytes = n.value, bool(c.value), b.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tsk_destroy(self.h)
            self.h = None

    @property
    def state_dtype(self):
        if self.is_complex:
            return torch.complex128
        return torch.float64 if self.elem_bytes == 8 else torch.float32

    def new_state(self, device="cuda"):
        return torch.zeros(self.n, dtype=self.state_dtype, device=device)


# ---- same-named wrappers of the C entry points ---------------------------------------------
def create_cgle1d(n=256, half_width=50.0, stream=None):
    h = C.c_void_p()
    _check(load().tsk_create_cgle1d(C.byref(h), n, half_width, _stream(stream)))
    return Op(h, "cgle1d")


def set_params_cgle(op, U, c_u, c_d, mu0, mu2, dt, T):
    _check(load().tsk_set_params_cgle(op.h, U, c_u, c_d, mu0, mu2, dt, T))


def create_kolmo2d(N, precision=TSK_FP64, stream=None):
    h = C.c_void_p()
    _check(load().tsk_create_kolmo2d(C.byref(h), N, precision, _stream(stream)))
    op = Op(h, "kolmo2d")
    op.N = N
    return op


def set_params_kolmo(op, Re, alpha, dt, T):
    _check(load().tsk_set_params_kolmo(op.h, Re, alpha, dt, T))


def set_base_parallel(op, U_y, dOmega_dy):
    a, pa = _dbl(U_y)
    b, pb = _dbl(dOmega_dy)
    if a.size != op.N or b.size != op.N:
        raise ValueError(f"base profiles must have N = {op.N} samples")
    _check(load().tsk_set_base_parallel(op.h, pa, pb))


def set_base_kolmogorov(op, n_forcing=4):
    _check(load().tsk_set_base_kolmogorov(op.h, n_forcing))


def set_base_flow(op, U, V, dOmega_dx, dOmega_dy):
    arrs = [_dbl(x) for x in (U, V, dOmega_dx, dOmega_dy)]
    if any(a.size != op.N * op.N for a, _ in arrs):
        raise ValueError(f"base fields must have N*N = {op.N * op.N} samples")
    _check(load().tsk_set_base_flow(op.h, *[p for _, p in arrs]))


def set_tuning(op, columns_per_wave):
    _check(load().tsk_set_tuning(op.h, int(columns_per_wave)))


def get_tuning(op):
    c = C.c_int()
    _check(load().tsk_get_tuning(op.h, C.byref(c)))
    return c.value


def set_stepper_waves(op, waves_per_group):
    _check(load().tsk_set_stepper_waves(op.h, int(waves_per_group)))


def get_stepper_waves(op):
    w = C.c_int()
    _check(load().tsk_get_stepper_waves(op.h, C.byref(w)))
    return w.value


def set_stop_rule(op, res_floor_rel=-1.0, dup_rel=-1.0):
    """Per-operator stop rule (tsk_set_stop_rule); negative values restore the
    defaults of the state type."""
    _check(load().tsk_set_stop_rule(op.h, float(res_floor_rel), float(dup_rel)))


def _phys_spec(op):
    if op.is_complex:
        return op.n, torch.complex128
    return op.N * op.N, op.state_dtype


def from_physical(op, phys, state):
    _need(phys, *_phys_spec(op), "physical field")
    _need(state, op.n, op.state_dtype, "state")
    _check(load().tsk_from_physical(op.h, _ptr(phys), _ptr(state)))


def to_physical(op, state, phys):
    _need(phys, *_phys_spec(op), "physical field")
    _need(state, op.n, op.state_dtype, "state")
    _check(load().tsk_to_physical(op.h, _ptr(state), _ptr(phys)))


def apply(op, x, y):
    _need(x, op.n, op.state_dtype, "x")
    _need(y, op.n, op.state_dtype, "y")
    _check(load().tsk_apply(op.h, _ptr(x), _ptr(y)))


def arnoldi(op, m, k, tol, v0=None, seed=0, want_vectors=False):
    """Run tsk_arnoldi; returns a dict with mu, lam (complex numpy), res, status,
    n_matvec, n_ritz, n_converged, beta, ms_total and X (Ritz vectors, complex128
    tensor n x k on the device) when want_vectors."""
    import numpy as np
    if v0 is not None:
        _need(v0, op.n, op.state_dtype, "v0")
    mu = np.zeros(2 * k)
    lam = np.zeros(2 * k)
    res = np.zeros(k)
    X = None
    if want_vectors:
        X = torch.zeros((k, op.n), dtype=torch.complex128, device="cuda")
    info = ArnoldiInfo()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    st = load().tsk_arnoldi(op.h, m, k, tol, _ptr(v0) if v0 is not None else None, C.c_uint64(seed),
                            pd(mu), pd(lam), pd(res), _ptr(X) if X is not None else None, C.byref(info))
    _check(st)
    nr = info.n_ritz
    out = dict(mu=(mu[0::2] + 1j * mu[1::2])[:nr], lam=(lam[0::2] + 1j * lam[1::2])[:nr], res=res[:nr],
               status=st, n_matvec=info.n_matvec, n_ritz=nr, n_converged=info.n_converged,
               beta=info.beta, ms_total=info.ms_total, ms_apply=info.ms_apply)
    if X is not None:
        out["X"] = X[:nr]
    return out


def batch_arnoldi(ops, m, k, tol, v0s=None, seeds=None, want_vectors=False):
    """Run tsk_batch_arnoldi on a list of operators (same state type and stream).
    Returns a list of dicts like ``arnoldi`` (X when want_vectors)."""
    import numpy as np
    count = len(ops)
    if v0s is not None:
        for op, v in zip(ops, v0s):
            if v is not None:
                _need(v, op.n, op.state_dtype, "v0")
    hs = (C.c_void_p * count)(*[op.h for op in ops])
    v0p = None
    if v0s is not None:
        v0p = (C.c_void_p * count)(*[(v.data_ptr() if v is not None else None) for v in v0s])
    sp = None
    if seeds is not None:
        sp = (C.c_uint64 * count)(*[int(x) for x in seeds])
    mu = np.zeros(2 * k * count)
    lam = np.zeros(2 * k * count)
    res = np.zeros(k * count)
    Xs = [torch.zeros((k, op.n), dtype=torch.complex128, device="cuda") for op in ops] if want_vectors else None
    rp = (C.c_void_p * count)(*[x.data_ptr() for x in Xs]) if Xs else None
    infos = (ArnoldiInfo * count)()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(load().tsk_batch_arnoldi(hs, count, m, k, tol, v0p, sp, pd(mu), pd(lam), pd(res), rp, infos))
    out = []
    for i in range(count):
        f = infos[i]
        nr = f.n_ritz
        o = dict(mu=(mu[2 * k * i:2 * k * (i + 1):2] + 1j * mu[2 * k * i + 1:2 * k * (i + 1):2])[:nr],
                 lam=(lam[2 * k * i:2 * k * (i + 1):2] + 1j * lam[2 * k * i + 1:2 * k * (i + 1):2])[:nr],
                 res=res[k * i:k * (i + 1)][:nr], status=f.status, n_matvec=f.n_matvec, n_ritz=nr,
                 n_converged=f.n_converged, beta=f.beta, ms_total=f.ms_total, ms_apply=f.ms_apply)
        if Xs:
            o["X"] = Xs[i][:nr]
        out.append(o)
    return out


def set_nonlinear(op, n_forcing=4, U0=0.0, extra_forcing=None):
    """Nonlinear forced equation on a Navier-Stokes operator (extra_forcing: N x N
    physical field or None)."""
    ex, exp_ = (None, None) if extra_forcing is None else _dbl(extra_forcing)
    if ex is not None and ex.size != op.N * op.N:
        raise ValueError("extra forcing must have N*N samples")
    _check(load().tsk_set_nonlinear(op.h, n_forcing, U0, exp_))


def laminar_state(op):
    x = op.new_state()
    _check(load().tsk_laminar_state(op.h, _ptr(x)))
    return x


def nonlinear_step(op, x, y, nsteps=0):
    _need(x, op.n, op.state_dtype, "x")
    _need(y, op.n, op.state_dtype, "y")
    _check(load().tsk_nonlinear_step(op.h, _ptr(x), _ptr(y), nsteps))


def set_base_from_state(op, x):
    _need(x, op.n, op.state_dtype, "x")
    _check(load().tsk_set_base_from_state(op.h, _ptr(x)))


def _fp_out(st, info, hist, n):
    return dict(status=st, iterations=info.iterations, time_steps=info.time_steps, basis_dim=info.basis_dim,
                residual=info.residual, ms_total=info.ms_total, hist=hist[:n].copy())


def sfd(op, x, chi, delta, check_every, tol, max_checks):
    """Selective frequency damping in place on the device state x."""
    import numpy as np
    _need(x, op.n, op.state_dtype, "x")
    hist = np.zeros(max_checks)
    info = FpInfo()
    st = load().tsk_sfd(op.h, _ptr(x), chi, delta, check_every, tol, max_checks,
                        hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(info))
    _check(st)
    return _fp_out(st, info, hist, info.iterations)


def rpm(op, x, m, k, delta, tol, max_iter):
    """Recursive projection method in place on the device state x."""
    import numpy as np
    _need(x, op.n, op.state_dtype, "x")
    hist = np.zeros(max_iter)
    info = FpInfo()
    st = load().tsk_rpm(op.h, _ptr(x), m, k, delta, tol, max_iter, hist.ctypes.data_as(C.POINTER(C.c_double)),
                        C.byref(info))
    _check(st)
    return _fp_out(st, info, hist, min(info.iterations + 1, max_iter))


def boostconv(op, x, m, tol, max_iter):
    """BoostConv in place on the device state x."""
    import numpy as np
    _need(x, op.n, op.state_dtype, "x")
    hist = np.zeros(max_iter)
    info = FpInfo()
    st = load().tsk_boostconv(op.h, _ptr(x), m, tol, max_iter, hist.ctypes.data_as(C.POINTER(C.c_double)),
                              C.byref(info))
    _check(st)
    return _fp_out(st, info, hist, min(info.iterations + 1, max_iter))


def set_resolvent(op, omega, t_transient):
    """Resolvent mode of a Ginzburg-Landau operator (t_transient = 0: propagator)."""
    _check(load().tsk_set_resolvent(op.h, omega, t_transient))


def apply_adjoint(op, x, y):
    """y = M^dagger x (device state tensors of the operator's dtype)."""
    _need(x, op.n, op.state_dtype, "x")
    _need(y, op.n, op.state_dtype, "y")
    _check(load().tsk_apply_adjoint(op.h, _ptr(x), _ptr(y)))


def optimal_perturbation(op, m, k, tol, v0=None, seed=0, want_vectors=False):
    """Run tsk_optimal_perturbation; returns a dict with sigma, gain (= sigma^2),
    res, status, n_steps, n_converged, ms_total, ms_apply and X (right singular
    vectors, complex128 k x n on the device) when want_vectors."""
    import numpy as np
    if v0 is not None:
        _need(v0, op.n, op.state_dtype, "v0")
    sig = np.zeros(k)
    res = np.zeros(k)
    X = torch.zeros((k, op.n), dtype=torch.complex128, device="cuda") if want_vectors else None
    info = ArnoldiInfo()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    st = load().tsk_optimal_perturbation(op.h, m, k, tol, _ptr(v0) if v0 is not None else None, C.c_uint64(seed),
                                         pd(sig), pd(res), _ptr(X) if X is not None else None, C.byref(info))
    _check(st)
    nr = info.n_ritz
    out = dict(sigma=sig[:nr], gain=sig[:nr] ** 2, res=res[:nr], status=st, n_steps=info.n_matvec, n_ritz=nr,
               n_converged=info.n_converged, beta=info.beta, ms_total=info.ms_total, ms_apply=info.ms_apply)
    if X is not None:
        out["X"] = X[:nr]
    return out


def batch_optimal_perturbation(ops, m, k, tol, v0s=None, seeds=None, want_vectors=False):
    """Run tsk_batch_optimal_perturbation on a list of operators (same state type
    and stream, each with an adjoint).  Returns a list of dicts like
    ``optimal_perturbation`` (X when want_vectors)."""
    import numpy as np
    count = len(ops)
    if v0s is not None:
        for op, v in zip(ops, v0s):
            if v is not None:
                _need(v, op.n, op.state_dtype, "v0")
    hs = (C.c_void_p * count)(*[op.h for op in ops])
    v0p = None
    if v0s is not None:
        v0p = (C.c_void_p * count)(*[(v.data_ptr() if v is not None else None) for v in v0s])
    sp = (C.c_uint64 * count)(*[int(x) for x in seeds]) if seeds is not None else None
    sig = np.zeros(k * count)
    res = np.zeros(k * count)
    Xs = [torch.zeros((k, op.n), dtype=torch.complex128, device="cuda") for op in ops] if want_vectors else None
    rp = (C.c_void_p * count)(*[x.data_ptr() for x in Xs]) if Xs else None
    infos = (ArnoldiInfo * count)()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(load().tsk_batch_optimal_perturbation(hs, count, m, k, tol, v0p, sp, pd(sig), pd(res), rp, infos))
    out = []
    for i in range(count):
        f = infos[i]
        nr = f.n_ritz
        sg = sig[k * i:k * (i + 1)][:nr]
        o = dict(sigma=sg, gain=sg ** 2, res=res[k * i:k * (i + 1)][:nr], status=f.status, n_steps=f.n_matvec,
                 n_ritz=nr, n_converged=f.n_converged, beta=f.beta, ms_total=f.ms_total, ms_apply=f.ms_apply)
        if Xs:
            o["X"] = Xs[i][:nr]
        out.append(o)
    return out


def krylov_schur(op, m, k, tol, delta=0.1, p_max=0, max_restarts=50, v0=None, seed=0, want_vectors=False):
    """Run tsk_krylov_schur; returns a dict like ``arnoldi`` plus n_restarts and
    kept_last."""
    import numpy as np
    if v0 is not None:
        _need(v0, op.n, op.state_dtype, "v0")
    mu = np.zeros(2 * k)
    lam = np.zeros(2 * k)
    res = np.zeros(k)
    X = None
    if want_vectors:
        X = torch.zeros((k, op.n), dtype=torch.complex128, device="cuda")
    info = KsInfo()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    st = load().tsk_krylov_schur(op.h, m, k, tol, delta, p_max, max_restarts,
                                 _ptr(v0) if v0 is not None else None, C.c_uint64(seed), pd(mu), pd(lam), pd(res),
                                 _ptr(X) if X is not None else None, C.byref(info))
    _check(st)
    nr = info.n_ritz
    out = dict(mu=(mu[0::2] + 1j * mu[1::2])[:nr], lam=(lam[0::2] + 1j * lam[1::2])[:nr], res=res[:nr],
               status=st, n_matvec=info.n_matvec, n_restarts=info.n_restarts, kept_last=info.kept_last,
               n_ritz=nr, n_converged=info.n_converged, beta=info.beta, ms_total=info.ms_total,
               ms_apply=info.ms_apply)
    if X is not None:
        out["X"] = X[:nr]
    return out


def batch_krylov_schur(ops, m, k, tol, delta=0.1, p_max=0, max_restarts=50, v0s=None, seeds=None,
                       want_vectors=False):
    """Run tsk_batch_krylov_schur on a list of real operators (same state type
    and stream).  Returns a list of dicts like ``krylov_schur`` (X when
    want_vectors)."""
    import numpy as np
    count = len(ops)
    if v0s is not None:
        for op, v in zip(ops, v0s):
            if v is not None:
                _need(v, op.n, op.state_dtype, "v0")
    hs = (C.c_void_p * count)(*[op.h for op in ops])
    v0p = None
    if v0s is not None:
        v0p = (C.c_void_p * count)(*[(v.data_ptr() if v is not None else None) for v in v0s])
    sp = None
    if seeds is not None:
        sp = (C.c_uint64 * count)(*[int(x) for x in seeds])
    mu = np.zeros(2 * k * count)
    lam = np.zeros(2 * k * count)
    res = np.zeros(k * count)
    Xs = [torch.zeros((k, op.n), dtype=torch.complex128, device="cuda") for op in ops] if want_vectors else None
    rp = (C.c_void_p * count)(*[x.data_ptr() for x in Xs]) if Xs else None
    infos = (KsInfo * count)()
    pd = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(load().tsk_batch_krylov_schur(hs, count, m, k, tol, delta, p_max, max_restarts, v0p, sp, pd(mu), pd(lam),
                                         pd(res), rp, infos))
    out = []
    for i in range(count):
        f = infos[i]
        nr = f.n_ritz
        o = dict(mu=(mu[2 * k * i:2 * k * (i + 1):2] + 1j * mu[2 * k * i + 1:2 * k * (i + 1):2])[:nr],
                 lam=(lam[2 * k * i:2 * k * (i + 1):2] + 1j * lam[2 * k * i + 1:2 * k * (i + 1):2])[:nr],
                 res=res[k * i:k * (i + 1)][:nr], status=f.status, n_matvec=f.n_matvec, n_restarts=f.n_restarts,
                 kept_last=f.kept_last, n_ritz=nr, n_converged=f.n_converged, beta=f.beta, ms_total=f.ms_total,
                 ms_apply=f.ms_apply)
        if Xs:
            o["X"] = Xs[i][:nr]
        out.append(o)
    return out


def ks_contract(H, beta, k, delta=0.1, p_max=0, stream=None):
    """Device Krylov-Schur contraction of an m x m real Hessenberg tensor (cuda).
    Returns (mu, res, Hnew ((p+1) x p), W (m x p), beta_new)."""
    m = H.shape[0]
    if H.dim() != 2 or H.shape[1] != m or not H.is_cuda:
        raise ValueError("H must be a square CUDA/HIP tensor")
    Hc = H.to(torch.float64).t().contiguous()  # column-major storage
    mu = torch.zeros(m, dtype=torch.complex128, device=H.device)
    res = torch.zeros(m, dtype=torch.float64, device=H.device)
    Hn = torch.zeros((m, m + 1), dtype=torch.float64, device=H.device)  # column-major (m+1) x m
    W = torch.zeros((m, m), dtype=torch.float64, device=H.device)     # column-major m x m
    kept, bnew = C.c_int(), C.c_double()
    _check(load().tsk_ks_contract(_ptr(Hc), m, m, beta, k, delta, p_max, _ptr(mu), _ptr(res), _ptr(Hn), _ptr(W),
                                  C.byref(kept), C.byref(bnew), _stream(stream)))
    p = kept.value
    return mu, res, Hn.t()[: p + 1, :p], W.t()[:, :p], bnew.value


def last_hessenberg(op):
    import numpy as np
    m, steps = C.c_int(), C.c_int()
    _check(load().tsk_last_hessenberg(op.h, None, C.byref(m), C.byref(steps)))
    buf = np.zeros(2 * (m.value + 1) * m.value)
    _check(load().tsk_last_hessenberg(op.h, buf.ctypes.data_as(C.POINTER(C.c_double)), C.byref(m),
                                      C.byref(steps)))
    H = (buf[0::2] + 1j * buf[1::2]).reshape(m.value, m.value + 1).T  # column-major
    s = steps.value
    return H[: s + 1, :s]


def last_basis(op):
    """Device basis of the last run as a tensor view (steps+1 rows)."""
    p, ld = C.c_void_p(), C.c_int64()
    _check(load().tsk_last_basis(op.h, C.byref(p), C.byref(ld)))
    return p.value, ld.value


def hessenberg_ritz(H, beta, stream=None):
    """Device eigensolve of a p x p complex128 Hessenberg tensor (cuda)."""
    p = H.shape[0]
    if H.dim() != 2 or H.shape[1] != p or not H.is_cuda:
        raise ValueError("H must be a square CUDA/HIP tensor")
    Hc = H.to(torch.complex128).t().contiguous()  # column-major storage
    mu = torch.zeros(p, dtype=torch.complex128, device=H.device)
    Y = torch.zeros((p, p), dtype=torch.complex128, device=H.device)
    res = torch.zeros(p, dtype=torch.float64, device=H.device)
    _check(load().tsk_hessenberg_ritz(_ptr(Hc), p, p, beta, _ptr(mu), _ptr(Y), _ptr(res), _stream(stream)))
    return mu, Y.t(), res  # Y rows were columns


def hessenberg_ritz_real(H, beta, stream=None):
    """Device real double-shift QR of a p x p real Hessenberg tensor (cuda):
    eigenvalues (complex128) and residual estimates beta |e_p^T y|."""
    p = H.shape[0]
    if H.dim() != 2 or H.shape[1] != p or not H.is_cuda:
        raise ValueError("H must be a square CUDA/HIP tensor")
    Hc = H.to(torch.float64).t().contiguous()  # column-major storage
    mu = torch.zeros(p, dtype=torch.complex128, device=H.device)
    res = torch.zeros(p, dtype=torch.float64, device=H.device)
    _check(load().tsk_hessenberg_ritz_real(_ptr(Hc), p, p, beta, _ptr(mu), _ptr(res), _stream(stream)))
    return mu, res


def hessenberg_ritz_real_noalloc(H_colmajor, ldh, p, beta, mu, res, stream=None):
    """tsk_hessenberg_ritz_real_noalloc on caller buffers: H_colmajor holds
    ldh * p doubles (column-major, leading dimension ldh), mu p complex128,
    res p doubles, all on the device.  Allocates nothing."""
    p, ldh = int(p), int(ldh)
    _need(H_colmajor, ldh * p, torch.float64, "H")
    _need(mu, p, torch.complex128, "mu")
    _need(res, p, torch.float64, "res")
    _check(load().tsk_hessenberg_ritz_real_noalloc(_ptr(H_colmajor), ldh, p, float(beta), _ptr(mu), _ptr(res),
                                                    _stream(stream)))


def normal_fill(count, seed, stream=None):
    count = int(count)
    if count < 0:
        raise ValueError("count must be >= 0")
    out = torch.zeros(count, dtype=torch.float64, device="cuda")
    _check(load().tsk_normal_fill(C.c_void_p(out.data_ptr()), count, C.c_uint64(seed), _stream(stream)))
    return out


# ---- learned start vector ------------------------------------------------------------------
MLP_OUT = 2048


class Mlp:
    """Owning wrapper of a tsk_mlp handle."""

    def __init__(self, handle, width):
        self.h = handle
        self.width = width
        n = C.c_int64()
        _check(load().tsk_mlp_param_count(self.h, C.byref(n)))
        self.param_count = n.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.tsk_mlp_destroy(self.h)
            self.h = None


def mlp_create(width=512, in_lo=(5.0, 0.25), in_hi=(40.0, 1.0), stream=None):
    h = C.c_void_p()
    lo, plo = _dbl(in_lo)
    hi, phi = _dbl(in_hi)
    if lo.size != 2 or hi.size != 2:
        raise ValueError("in_lo and in_hi hold (Re, alpha)")
    _check(load().tsk_mlp_create(C.byref(h), int(width), plo, phi, _stream(stream)))
    return Mlp(h, int(width))


def mlp_init(net, seed):
    _check(load().tsk_mlp_init(net.h, C.c_uint64(seed)))


def mlp_set_params(net, params):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != net.param_count:
        raise ValueError(f"expected {net.param_count} parameters, got {a.size}")
    _check(load().tsk_mlp_set_params(net.h, C.c_void_p(a.ctypes.data)))


def mlp_get_params(net):
    import numpy as np
    a = np.zeros(net.param_count, dtype=np.float32)
    _check(load().tsk_mlp_get_params(net.h, C.c_void_p(a.ctypes.data)))
    return a


def _batch_inputs(inputs):
    if not isinstance(inputs, torch.Tensor) or not inputs.is_cuda or inputs.dtype != torch.float32 \
            or inputs.dim() != 2 or inputs.shape[1] != 2 or not inputs.is_contiguous():
        raise ValueError("inputs: contiguous float32 CUDA/HIP tensor of shape (batch, 2) holding (Re, alpha)")
    return inputs.shape[0]


def mlp_forward(net, inputs):
    B = _batch_inputs(inputs)
    out = torch.empty((B, MLP_OUT), dtype=torch.float32, device=inputs.device)
    _check(load().tsk_mlp_forward(net.h, _ptr(inputs), B, _ptr(out)))
    return out


def mlp_gradients(net, inputs, targets):
    B = _batch_inputs(inputs)
    _need(targets, B * MLP_OUT, torch.float32, "targets")
    grad = torch.empty(net.param_count, dtype=torch.float32, device=inputs.device)
    loss = C.c_double()
    _check(load().tsk_mlp_gradients(net.h, _ptr(inputs), _ptr(targets), B, _ptr(grad), C.byref(loss)))
    return grad, loss.value


def mlp_train(net, inputs, targets, steps, lr):
    import numpy as np
    B = _batch_inputs(inputs)
    _need(targets, B * MLP_OUT, torch.float32, "targets")
    losses = np.zeros(int(steps))
    _check(load().tsk_mlp_train(net.h, _ptr(inputs), _ptr(targets), B, int(steps), float(lr),
                                losses.ctypes.data_as(C.POINTER(C.c_double))))
    return losses


def ritz_block_target(op, ritz, use=None):
    """Training target (2048 float32 on the device) from Ritz vectors (k x n
    complex128 tensor, as returned by arnoldi(..., want_vectors=True))."""
    if ritz.dim() != 2 or ritz.shape[1] != op.n:
        raise ValueError("ritz: (k, n) complex128 tensor")
    k = ritz.shape[0]
    _need(ritz, k * op.n, torch.complex128, "ritz")
    up = None
    if use is not None:
        if len(use) != k:
            raise ValueError("use: one flag per Ritz vector")
        up = (C.c_int * k)(*[1 if u else 0 for u in use])
    out = torch.empty(MLP_OUT, dtype=torch.float32, device=ritz.device)
    _check(load().tsk_ritz_block_target(op.h, _ptr(ritz), k, up, _ptr(out)))
    return out


def mlp_start(net, op, Re, alpha, gamma=0.1, seed=0):
    """Learned start vector for op at (Re, alpha); returns (state tensor, used_net)."""
    v0 = op.new_state()
    used = C.c_int()
    _check(load().tsk_mlp_start(net.h, op.h, float(Re), float(alpha), float(gamma), C.c_uint64(seed),
                                _ptr(v0), C.byref(used)))
    return v0, bool(used.value)
