"""Writes the stored oracle results used by the GPU parity tests at full size.

Calls only ``oracle/`` (and the seeded input generators of ``workloads``); no
value comes from the HIP path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.arnoldi import arnoldi  # noqa: E402
from oracle.cgle import CGLE  # noqa: E402
from oracle.kolmogorov import Kolmogorov  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _pack(r):
    return dict(n_matvec=int(r["n_matvec"]), status=int(r["status"]),
                lam_re=[float(x.real) for x in r["lam"]], lam_im=[float(x.imag) for x in r["lam"]],
                mu_re=[float(x.real) for x in r["mu"]], mu_im=[float(x.imag) for x in r["mu"]],
                res=[float(x) for x in r["res"]])


def kolmo128():
    c = W.KOLMO_128_FP64
    op = Kolmogorov.kolmogorov(c["N"], c["alpha"], c["Re"], c["dt"], c["T"], c["n_forcing"])
    N = c["N"]
    v0 = op.project(W.kolmo_start_physical(N, 0)).ravel()
    r = arnoldi(lambda v: op.apply(v.reshape(N, N)).ravel(), v0, c["m"], c["k"], c["tol"], T=c["T"],
                keep_basis=False)
    d = _pack(r)
    d["workload"] = "kolmogorov N=128 fp64, start = projected N(0,1) field workloads.kolmo_start_physical(128, 0)"
    return d


def kolmo128_m53():
    """The 128^2 FP64 operator at a fixed order: m = 53 Arnoldi steps (the
    order at which six distinct pairs first reach 1e-8), tol = 0 so every
    step runs, k = 12 wanted values, with every Ritz value of H_53."""
    c = W.KOLMO_128_FP64
    op = Kolmogorov.kolmogorov(c["N"], c["alpha"], c["Re"], c["dt"], c["T"], c["n_forcing"])
    N = c["N"]
    v0 = op.project(W.kolmo_start_physical(N, 0)).ravel()
    r = arnoldi(lambda v: op.apply(v.reshape(N, N)).ravel(), v0, 53, 12, 0.0, T=c["T"], keep_basis=False)
    d = _pack(r)
    H = r["H"][:53, :53].real
    ev, vr = np.linalg.eig(H)
    beta = abs(r["H"][53, 52])
    res = beta * np.abs(vr[-1, :]) / np.linalg.norm(vr, axis=0)
    lam = np.log(ev.astype(complex)) / c["T"]
    d["all_lam_re"] = [float(x.real) for x in lam]
    d["all_lam_im"] = [float(x.imag) for x in lam]
    d["all_res"] = [float(x) for x in res]
    d["workload"] = ("kolmogorov N=128 fp64, m=53 k=12 tol=0, start = projected N(0,1) field "
                     "workloads.kolmo_start_physical(128, 0)")
    return d


def cgle256():
    c = W.CGLE
    op = CGLE(n=c["n"], half_width=c["half_width"], U=c["U"], c_u=c["c_u"], c_d=c["c_d"], mu0=c["mu0"],
              mu2=c["mu2"], dt=c["dt"], T=c["T"])
    r = arnoldi(op.apply, W.cgle_start(c["n"], 0), c["m"], c["k"], c["tol"], T=c["T"], keep_basis=False)
    d = _pack(r)
    d["workload"] = "cgle n=256, start = workloads.cgle_start(256, 0)"
    return d


JOBS = (("oracle_cgle256.json", cgle256), ("oracle_kolmo128_fp64.json", kolmo128),
        ("oracle_kolmo128_fp64_m53.json", kolmo128_m53))

if __name__ == "__main__":
    only = sys.argv[1:]
    for name, fn in JOBS:
        if only and name not in only:
            continue
        d = fn()
        with open(os.path.join(OUT, name), "w") as f:
            json.dump(d, f, indent=1)
        print(name, d["n_matvec"], d["status"])
