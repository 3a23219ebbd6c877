"""Benchmark of the time-stepper Arnoldi path on one MI355X.

Default workload (--workload learned): wall time to 6 Ritz pairs on 16 held-out
linearized Kolmogorov flows at 256 x 256 (Re ~ U[5, 40], alpha in {0.25, 0.5,
0.75, 1}; IF-RK4 dt = 0.005, T = 1; Arnoldi m = 96, k = 6, tol = 1e-8), for the
FP32 precision form with the learned start vector against the plain FP64 form
with a seeded random start (and two more forms for an equal-accuracy view).
A step is one solve of each of the 16 instances in each form; a solve is one
whole tsk_arnoldi call: start vector, a matvec (200 IF-RK4 steps) per Krylov
vector, CGS2, the device Hessenberg QR and stop test after every matvec, and the
Ritz values and vectors at the end.  The network is trained first (untimed).
The line also carries the 64-instance sweep's throughput, the accuracy of every
form (true residuals by an FP64 matvec, |dlambda| against FP64), the roofline
of the dominant kernel and the CPU oracle's time on the same operator.

Other workloads: kolmo128 (128^2 FP64), kolmo256-fp32, kolmo512-fp32, sweep, cgle, general,
krylov-schur, optimal, fixed-point, resolvent, copy.

Prints ONE JSON line (rank 0).  Other output goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X published FP64 vector peak
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak


def colstep_flops(N, nsteps):
    """Algorithmic flops of one matvec of the column stepper: per dealiased
    column kx >= 1 and RK stage, one inverse and one forward complex FFT of length
    N (5 N log2 N each), the product with the base profile (2 N) and the
    spectral bookkeeping (12 flops per kept mode)."""
    M = (N - 1) // 3
    NM = 2 * M + 1
    per_stage = 2 * 5 * N * math.log2(N) + 2 * N + 12 * NM
    return M * 4 * nsteps * per_stage


def bloch_flops(N, nsteps, sectors=4):
    """Algorithmic flops of one matvec of the Bloch-sector stepper: per dealiased
    column kx >= 1 and RK stage, in each of the four sectors one inverse and one
    forward complex FFT of length N/4 (5 L log2 L each), the product with the
    base profile (2 flops per grid point) and the spectral bookkeeping (12 flops
    per kept mode)."""
    M = (N - 1) // 3
    NM = 2 * M + 1
    L = N // sectors
    per_stage = sectors * 2 * 5 * L * math.log2(L) + 2 * N + 12 * NM
    return M * 4 * nsteps * per_stage


def couple_flops(N, nsteps, nh=4):
    """Algorithmic flops of one matvec of the spectral-coupling stepper: per kept
    mode of the columns kx >= 1 (complex) and IF-RK4 step, four stages of the
    coupling factor (2) and the neighbour difference (2), the Lawson updates
    (4 + 4 + 4 + 2 complex fused multiply-adds = 28) and the two scaled copies
    of the step's input (4): 48; the kx = 0 column decays (2 per mode and step)."""
    M = (N - 1) // 3
    return nsteps * (48 * M * (2 * M + 1) + 2 * M)


def stepper_flops(tsk, op, N, nsteps):
    """Flop model and kernel name of the stepper the operator's matvec runs."""
    t = tsk.get_tuning(op)
    rt = "double" if op.elem_bytes == 8 else "float"
    if t == -2:
        M = (N - 1) // 3
        return couple_flops(N, nsteps), f"k_colstep_couple<{rt},{1 if (2 * M + 1 + 3) // 4 <= 64 else 2}>"
    if t == -1:
        return bloch_flops(N, nsteps), (f"k_colstep_bloch_split<{rt}>" if N == 128 else
                                        f"k_colstep_bloch<{rt},{N // 4}>")
    return colstep_flops(N, nsteps), f"k_colstep<{rt},{N},true>"


def cpu_baseline(seconds=12.0):
    """The CPU oracle (NumPy FP64, single thread) on a bounded sample of the same
    workload: as many full matvecs (200 IF-RK4 steps each) of the 128^2 operator
    as fit in about `seconds`."""
    import numpy as np  # noqa: F401

    import workloads as W
    from oracle.kolmogorov import Kolmogorov
    c = W.KOLMO_128_FP64
    N = c["N"]
    op = Kolmogorov.kolmogorov(N, c["alpha"], c["Re"], c["dt"], c["T"], c["n_forcing"])
    w = op.project(W.kolmo_start_physical(N, 0))
    t0 = time.perf_counter()
    count = 0
    while True:
        w = op.apply(w)
        w /= np.linalg.norm(w)
        count += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    tsgp = count * op.nsteps * N * N / el
    model, ncpu = cpu_model()
    return {"value": tsgp, "unit": "time-steps*gridpoints/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_logical_cores": ncpu,
            "sample": f"{count} oracle matvecs (200 IF-RK4 steps each) of the 128x128 FP64 operator, "
                      f"{el:.1f} s, NumPy/pocketfft single thread"}


COLSTEP_SOURCES = ("common.hpp", "colstep.hpp", "colcouple.hpp")
GENERAL_SOURCES = ("common.hpp", "fft.hpp", "kolmo2d.hip")


def measured_traffic(profile_name, sources=COLSTEP_SOURCES, key="traffic_bytes_per_launch"):
    """HBM bytes (per launch, or per `key`) from a committed rocprofv3 PMC
    summary, or None when the kernel sources changed since the counters were
    taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] in ("source_hash", key):
            rec[parts[0]] = parts[1]
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_1804_03859_amd", "csrc", f), "rb").read())
    if rec.get("source_hash") != h.hexdigest()[:16] or key not in rec:
        return None
    return float(rec[key])


def run_sweep(args, tsk, W, np, torch):
    """Batched neutral-curve sweep: 64 FP32 instances of mixed size in lockstep."""
    sweep = W.batch_sweep(64, 0)
    ops = []
    for c in sweep:
        op = tsk.create_kolmo2d(c["N"], tsk.TSK_FP32)
        tsk.set_params_kolmo(op, c["Re"], c["alpha"], c["dt"], c["T"])
        tsk.set_base_kolmogorov(op, c["n_forcing"])
        ops.append(op)
    phys = [torch.from_numpy(W.kolmo_start_physical(c["N"], i)).float().cuda().reshape(-1)
            for i, c in enumerate(sweep)]
    xs = [op.new_state() for op in ops]

    def step():
        for op, p_, x in zip(ops, phys, xs):
            tsk.from_physical(op, p_, x)
        return tsk.batch_krylov_schur(ops, 64, 4, 1e-8, delta=0.1, v0s=xs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rb = res[-1]
    ms = el * 1e3 / args.steps
    nsteps = int(round(sweep[0]["T"] / sweep[0]["dt"]))
    tsgp = sum(b["n_matvec"] * nsteps * c["N"] ** 2 for b, c in zip(rb, sweep))
    # every lockstep Arnoldi step launches the batched matvec of the instances still
    # active; ms_apply sums the HIP-event durations of those launches (the restart
    # cycles run as captured graphs, not timed per matvec).  Flops: each instance's
    # own matvecs of that phase (at most m = 64).
    ms_apply = rb[0]["ms_apply"]
    # every instance of this base runs the spectral-coupling stepper, all grid sizes in one launch
    flops_total = sum(min(b["n_matvec"], 64) * stepper_flops(tsk, op, c["N"], nsteps)[0]
                      for b, c, op in zip(rb, sweep, ops))
    achieved = flops_total / (ms_apply / 1e3) / 1e12
    return {
        "metric": "time-steps*gridpoints/s (batched neutral-curve sweep, all instances to 4 Ritz pairs at 1e-8, "
                  "batched Krylov-Schur restarts for those not converged at order 64)",
        "value": tsgp / (ms / 1e3), "unit": "time-steps*gridpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 Kolmogorov instances (24x128^2, 20x256^2, 20x384^2), FP32, Re~U[5,40], "
                               "alpha in {0.25,0.5,0.75,1}, m=64, k=4, tol=1e-8",
                   "n_matvec": [b["n_matvec"] for b in rb], "status": [b["status"] for b in rb],
                   "restarts": [b["n_restarts"] for b in rb],
                   "batched_matvec_ms_total": ms_apply},
        "roofline": {"bound": "alu", "kernel": "k_colstep_couple<float,1> (one batched matvec of all active instances)",
                     "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "matvec_ms_total": ms_apply,
                     "flops_total": flops_total, "traffic": None},
        "cpu_baseline": None,
    }


def run_single(args, tsk, W, np, torch, cfg, prec, dtype_name):
    N, m, k, tol = cfg["N"], cfg["m"], cfg["k"], cfg["tol"]
    nsteps = int(round(cfg["T"] / cfg["dt"]))
    op = tsk.create_kolmo2d(N, prec)
    tsk.set_params_kolmo(op, cfg["Re"], cfg["alpha"], cfg["dt"], cfg["T"])
    tsk.set_base_kolmogorov(op, cfg["n_forcing"])
    tdt = torch.float64 if prec == tsk.TSK_FP64 else torch.float32
    phys = torch.from_numpy(W.kolmo_start_physical(N, 0)).to(tdt).cuda().reshape(-1)
    x = op.new_state()

    def step():
        tsk.from_physical(op, phys, x)
        return tsk.arnoldi(op, m, k, tol, v0=x, want_vectors=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    r = results[-1]
    nmv = r["n_matvec"]
    tsgp_step = nmv * nsteps * N * N
    ms_apply = sum(q["ms_apply"] for q in results) / args.steps
    launch_ms = ms_apply / nmv
    stepper = tsk.get_tuning(op)  # -2 spectral coupling, -1 Bloch sectors, else columns per wavefront
    flops, kernel = stepper_flops(tsk, op, N, nsteps)
    traffic = None
    wkey = f"traffic_bytes_per_launch_w{tsk.get_stepper_waves(op)}"  # the launch shape the library kept
    if stepper == -2 and prec == tsk.TSK_FP64 and N == 128:
        traffic = measured_traffic("k_colstep_couple_kolmo128_fp64_hbm_traffic.md", key=wkey)
    elif stepper == -2 and prec == tsk.TSK_FP32 and N == 256:
        traffic = measured_traffic("k_colstep_couple_kolmo256_fp32_hbm_traffic.md", key=wkey)
    achieved = flops / (launch_ms / 1e3) / 1e12
    peak = FP64_VECTOR_PEAK_TFLOPS if prec == tsk.TSK_FP64 else FP32_VECTOR_PEAK_TFLOPS
    return {
        "metric": "time-steps*gridpoints/s (whole Arnoldi run to 6 Ritz pairs at residual 1e-8)",
        "value": tsgp_step / (ms_per_step / 1e3),
        "unit": "time-steps*gridpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": f"linearized Kolmogorov flow {N}x{N} {dtype_name.upper()}, Re=20, alpha=0.5, "
                               f"IF-RK4 dt=0.005 T=1, Arnoldi m={m} k={k} tol=1e-8, seeded N(0,1) start",
                   "n_matvec": nmv, "status": r["status"],
                   "stepper": {-2: "spectral coupling", -1: "bloch sectors"}.get(stepper,
                                                                                 f"{stepper} column(s) per wavefront"),
                   "wall_time_to_6_pairs_s": ms_per_step / 1e3,
                   "time_stepper_tsgp_per_s": tsgp_step / (ms_apply / 1e3),
                   "lambda": [round(float(v.real), 10) for v in r["lam"]],
                   "max_residual": float(np.max(r["res"]))},
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "launch_ms": launch_ms, "flops_per_launch": flops, "traffic": traffic},
        "cpu_baseline": None,
    }


def run_krylov_schur(args, tsk, W, np, torch):
    """Krylov-Schur (Sec. 3.2.2) on the 128^2 FP64 Kolmogorov operator with half
    the Arnoldi subspace (k_dim = 32, delta = 0.1, p_max = 16): a step is one whole
    restarted run to 6 Ritz pairs at residual 1e-8 from the seeded start.  The
    config also lists the matvec counts for other subspace sizes and for plain
    Arnoldi with m = 64 (untimed, one run each), like the paper's Table 1."""
    cfg = W.KOLMO_128_FP64
    N, k, tol = cfg["N"], cfg["k"], cfg["tol"]
    kdim, delta = 32, 0.1
    nsteps = int(round(cfg["T"] / cfg["dt"]))
    op = tsk.create_kolmo2d(N, tsk.TSK_FP64)
    tsk.set_params_kolmo(op, cfg["Re"], cfg["alpha"], cfg["dt"], cfg["T"])
    tsk.set_base_kolmogorov(op, cfg["n_forcing"])
    phys = torch.from_numpy(W.kolmo_start_physical(N, 0)).cuda().reshape(-1)
    x = op.new_state()

    def run(m, arnoldi=False):
        tsk.from_physical(op, phys, x)
        if arnoldi:
            return tsk.arnoldi(op, m, k, tol, v0=x, want_vectors=True)
        return tsk.krylov_schur(op, m, k, tol, delta=delta, v0=x, want_vectors=True)

    for _ in range(args.warmup):
        run(kdim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run(kdim) for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    r = results[-1]
    nmv = r["n_matvec"]
    tsgp_step = nmv * nsteps * N * N
    ms_apply = sum(q["ms_apply"] for q in results) / args.steps
    launch_ms = ms_apply / nmv
    flops, kname = stepper_flops(tsk, op, N, nsteps)
    achieved = flops / (launch_ms / 1e3) / 1e12
    table = {}
    for m in (16, 24, 48):
        q = run(m)
        table[f"krylov_schur_m{m}"] = {"n_matvec": q["n_matvec"], "restarts": q["n_restarts"],
                                       "status": q["status"], "ms": round(q["ms_total"], 2)}
    a = run(64, arnoldi=True)
    table["arnoldi_m64"] = {"n_matvec": a["n_matvec"], "status": a["status"], "ms": round(a["ms_total"], 2)}
    return {
        "metric": "time-steps*gridpoints/s (whole Krylov-Schur run to 6 Ritz pairs at residual 1e-8)",
        "value": tsgp_step / (ms_per_step / 1e3),
        "unit": "time-steps*gridpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"linearized Kolmogorov flow {N}x{N} FP64, Re=20, alpha=0.5, IF-RK4 dt=0.005 T=1, "
                               f"Krylov-Schur k_dim={kdim} delta={delta} p_max={kdim // 2} k={k} tol=1e-8, "
                               "seeded N(0,1) start",
                   "n_matvec": nmv, "n_restarts": r["n_restarts"], "status": r["status"],
                   "wall_time_to_6_pairs_s": ms_per_step / 1e3,
                   "time_stepper_tsgp_per_s": tsgp_step / (ms_apply / 1e3),
                   "non_matvec_ms": ms_per_step - ms_apply,
                   "lambda": [round(float(v.real), 10) for v in r["lam"]],
                   "max_residual": float(np.max(r["res"])), "subspace_table": table},
        "roofline": {"bound": "alu", "kernel": kname,
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "launch_ms": launch_ms, "flops_per_launch": flops,
                     "traffic": None},
        "cpu_baseline": None,
    }


def run_optimal(args, tsk, W, np, torch):
    """Optimal perturbation (Sec. 2.3.1 SVD formulation, Sec. 3.3.2) of the 128^2
    FP64 Kolmogorov propagator over T = 1: Lanczos on M^T M (each step one forward
    and one adjoint integration) to the 2 leading singular values at residual
    1e-8.  A step is one whole run from the seeded start.  The config also lists
    the optimal gain sigma_1^2 over other target times (untimed, one run each)."""
    cfg = W.KOLMO_128_FP64
    N, tol, m, k = cfg["N"], cfg["tol"], 40, 2
    nsteps = int(round(cfg["T"] / cfg["dt"]))

    def make(T):
        op = tsk.create_kolmo2d(N, tsk.TSK_FP64)
        tsk.set_params_kolmo(op, cfg["Re"], cfg["alpha"], cfg["dt"], T)
        tsk.set_base_kolmogorov(op, cfg["n_forcing"])
        return op

    op = make(cfg["T"])
    phys = torch.from_numpy(W.kolmo_start_physical(N, 0)).cuda().reshape(-1)
    x = op.new_state()

    def run(o):
        xx = o.new_state()
        tsk.from_physical(o, phys, xx)
        return tsk.optimal_perturbation(o, m, k, tol, v0=xx, want_vectors=True)

    for _ in range(args.warmup):
        run(op)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run(op) for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    r = results[-1]
    nint = 2 * r["n_steps"]  # integrations: forward + adjoint per Lanczos step
    tsgp_step = nint * nsteps * N * N
    ms_apply = sum(q["ms_apply"] for q in results) / args.steps
    launch_ms = ms_apply / nint
    # forward integrations by the operator's stepper, adjoint ones by its transpose: the transposed
    # coupling stepper does the same arithmetic per chain as the forward one; the transposed column
    # stepper (other stepper choices) has the column stepper's flops.  Flops averaged over the two kinds
    fwd_flops, fwd_kernel = stepper_flops(tsk, op, N, nsteps)
    coupled = tsk.get_tuning(op) == -2
    adj_flops = fwd_flops if coupled else colstep_flops(N, nsteps)
    adj_kernel = (fwd_kernel.replace("k_colstep_couple", "k_colstep_couple_adj") if coupled
                  else f"k_colstep_adj<double,{N},true>")
    flops = 0.5 * (fwd_flops + adj_flops)
    achieved = flops / (launch_ms / 1e3) / 1e12
    gains = {}
    for T in (0.25, 0.5, 2.0, 4.0):
        q = run(make(T))
        gains[f"T={T}"] = {"gain": float(q["gain"][0]), "sigma1": float(q["sigma"][0]), "steps": q["n_steps"]}
    gains[f"T={cfg['T']}"] = {"gain": float(r["gain"][0]), "sigma1": float(r["sigma"][0]), "steps": r["n_steps"]}
    del x
    return {
        "metric": "time-steps*gridpoints/s (whole optimal-perturbation run: Lanczos on M^T M to 2 singular values "
                  "at residual 1e-8)",
        "value": tsgp_step / (ms_per_step / 1e3),
        "unit": "time-steps*gridpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"optimal perturbation of the linearized Kolmogorov flow {N}x{N} FP64, Re=20, "
                               f"alpha=0.5, IF-RK4 dt=0.005, T=1, Lanczos m={m} k={k} tol=1e-8, seeded N(0,1) start",
                   "lanczos_steps": r["n_steps"], "integrations": nint, "status": r["status"],
                   "sigma": [float(v) for v in r["sigma"]], "gain": [float(v) for v in r["gain"]],
                   "max_residual": float(np.max(r["res"])),
                   "time_stepper_tsgp_per_s": tsgp_step / (ms_apply / 1e3), "gain_curve": gains},
        "roofline": {"bound": "alu", "kernel": fwd_kernel + " + " + adj_kernel,
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "launch_ms": launch_ms, "flops_per_launch": flops,
                     "traffic": None},
        "cpu_baseline": None,
    }


def general_stage_bytes(N, s):
    """Algorithmic HBM bytes of one RK4 stage of the general base-flow pipeline
    (s bytes per real): the row kernel reads the four derived fields G
    (4 x (M+1) x N complex) and the four base fields (4 N^2 reals) and writes the
    product spectrum Q ((M+1) x N complex); the column kernel reads Q, reads and
    writes the packed state and RK4 accumulator (n reals each) and writes G."""
    M = (N - 1) // 3
    n = 4 * M * (M + 1)
    g = 4 * (M + 1) * N * 2 * s
    q = (M + 1) * N * 2 * s
    row = g + 4 * N * N * s + q
    col = q + g + 4 * n * s
    return row, col


def run_fixed_point(args, tsk, W, np, torch):
    """Fixed points of the nonlinear forced Navier-Stokes equation (Sec. 3.1) on a
    128^2 FP64 grid: Re = 7, alpha = 0.5, drift U0 = 0.7 (three weakly unstable
    travelling modes), a weak two-dimensional extra forcing (so the fixed point has
    no analytic form), IF-RK4 dt = 0.02, outer iteration G = 100 steps (T = 2).
    A step is one whole RPM run (k_dim 24, delta 0.3) from the laminar flow to
    residual 1e-9; the config also reports BoostConv (m = 10) and SFD (chi = 0.2,
    omega_c = 0.2) on the same problem (untimed, one run each), like the paper's
    comparison of the three solvers."""
    N, Re, alpha, dt, T, U0 = 128, 7.0, 0.5, 0.02, 2.0, 0.7
    ex = W.random_forcing_field(N, alpha, 2, 7, 0.002)
    op = tsk.create_kolmo2d(N, tsk.TSK_FP64)
    tsk.set_params_kolmo(op, Re, alpha, dt, T)
    tsk.set_base_kolmogorov(op, 4)
    tsk.set_nonlinear(op, 4, U0, ex)
    tol = 1e-9

    def rpm_run():
        x = tsk.laminar_state(op)
        return x, tsk.rpm(op, x, 24, 1, 0.3, tol, 80)

    for _ in range(args.warmup):
        rpm_run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [rpm_run() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    xr, r = runs[-1]
    # time-stepper throughput and roofline: one nonlinear G (100 steps) timed alone
    y = op.new_state()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tsk.nonlinear_step(op, xr, y, 0)
    ev0.record()
    for _ in range(5):
        tsk.nonlinear_step(op, xr, y, 0)
    ev1.record()
    torch.cuda.synchronize()
    g_ms = ev0.elapsed_time(ev1) / 5
    nsteps = int(round(T / dt))
    row, col = general_stage_bytes(N, 8)
    row -= 4 * N * N * 8  # the nonlinear products read no base fields
    bytes_g = 4 * nsteps * (row + col)
    achieved = bytes_g / (g_ms / 1e3) / 1e9
    xb = tsk.laminar_state(op)
    b = tsk.boostconv(op, xb, 10, tol, 120)
    xs = tsk.laminar_state(op)
    sf = tsk.sfd(op, xs, 0.2, 5.0, 100, 1e-7, 400)
    agree = float(torch.linalg.norm(xr - xb).item() / torch.linalg.norm(xr).item())
    lam = tsk.laminar_state(op)
    dist = float(torch.linalg.norm(xr - lam).item() / torch.linalg.norm(lam).item())
    steps_rpm = r["time_steps"] + 24 * nsteps  # plus the Arnoldi factorisation of the Jacobian (24 matvecs)
    return {
        "metric": "time-steps*gridpoints/s (whole RPM fixed-point run to residual 1e-9)",
        "value": steps_rpm * N * N / (ms_per_step / 1e3),
        "unit": "time-steps*gridpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fixed point of the forced 2-D Navier-Stokes equation (Kolmogorov forcing n=4 + "
                               "band-limited extra forcing, amplitude 0.002, seed 7), 128x128 FP64, Re=7, alpha=0.5, "
                               "drift U0=0.7, IF-RK4 dt=0.02, G = 100 steps",
                   "rpm": {"iterations": r["iterations"], "basis_dim": r["basis_dim"], "residual": r["residual"],
                           "time_steps_incl_arnoldi": steps_rpm, "ms": ms_per_step},
                   "boostconv": {"iterations": b["iterations"], "residual": b["residual"],
                                 "time_steps": b["time_steps"], "ms": b["ms_total"], "status": b["status"]},
                   "sfd": {"checks": sf["iterations"], "residual_per_dt": sf["residual"],
                           "time_steps": sf["time_steps"], "ms": sf["ms_total"], "status": sf["status"]},
                   "rpm_vs_boostconv_rel_diff": agree, "fixed_point_distance_from_laminar_rel": dist,
                   "ms_per_G": g_ms},
        "roofline": {"bound": "hbm", "kernel": "k_gen_row<double,128,ROW_NL> + k_gen_col<double,128> (nonlinear step)",
                     "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "bytes_per_G": bytes_g, "traffic": None},
        "cpu_baseline": None,
    }


def run_general(args, tsk, W, np, torch):
    """Arnoldi on a general two-dimensional base flow (random band-limited base
    streamfunction, |jx|, |jy| <= 2, amplitude 0.3, seed 0), 128^2 FP64, through
    the full 2-D pseudo-spectral pipeline."""
    c = dict(W.KOLMO_128_FP64)
    N, m, k, tol = c["N"], c["m"], c["k"], c["tol"]
    nsteps = int(round(c["T"] / c["dt"]))
    op = tsk.create_kolmo2d(N, tsk.TSK_FP64)
    tsk.set_params_kolmo(op, c["Re"], c["alpha"], c["dt"], c["T"])
    tsk.set_base_flow(op, *W.random_base_fields(N, c["alpha"], 2, 0))
    phys = torch.from_numpy(W.kolmo_start_physical(N, 0)).cuda().reshape(-1)
    x = op.new_state()

    def step():
        tsk.from_physical(op, phys, x)
        return tsk.arnoldi(op, m, k, tol, v0=x)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    r = results[-1]
    nmv = r["n_matvec"]
    ms_apply = sum(q["ms_apply"] for q in results) / args.steps
    row, col = general_stage_bytes(N, 8)
    bytes_per_matvec = 4 * nsteps * (row + col) + 2 * op.n * 8
    achieved = bytes_per_matvec / (ms_apply / nmv / 1e3) / 1e9
    tsgp = nmv * nsteps * N * N
    stage_traffic = measured_traffic("general_base_128_fp64_trace_and_traffic.md", GENERAL_SOURCES,
                                     "traffic_bytes_per_stage")
    return {
        "metric": "time-steps*gridpoints/s (whole Arnoldi run to 6 Ritz pairs at residual 1e-8)",
        "value": tsgp / (ms / 1e3), "unit": "time-steps*gridpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "linearized Navier-Stokes about a random band-limited 2-D base flow (|j| <= 2, "
                               "amplitude 0.3, seed 0), 128x128 FP64, Re=20, alpha=0.5, IF-RK4 dt=0.005 T=1, "
                               "Arnoldi m=64 k=6 tol=1e-8, full 2-D pseudo-spectral pipeline",
                   "n_matvec": nmv, "status": r["status"], "ms_per_matvec": ms_apply / nmv,
                   "lambda": [[round(float(v.real), 10), round(float(v.imag), 10)] for v in r["lam"]]},
        "roofline": {"bound": "hbm", "kernel": "k_gen_row<double,128> + k_gen_col<double,128> (time stepper)",
                     "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "bytes_per_matvec": bytes_per_matvec,
                     "traffic": None if stage_traffic is None else stage_traffic * 4 * nsteps},
        "cpu_baseline": None,
    }


def cpu_model():
    """CPU model name of this host (from /proc/cpuinfo) and its logical core count."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline_learned(N, mean_matvecs, seconds=15.0):
    """The CPU oracle (NumPy FP64, single thread) on a bounded sample of the
    headline workload: whole matvecs (200 IF-RK4 steps each) of the first
    held-out 256^2 operator for about `seconds`; the per-matvec time times the
    FP64 form's mean matvec count gives the oracle's time per solve (its
    Hessenberg and Gram-Schmidt work is below 1% of that)."""
    import workloads as W
    from oracle.kolmogorov import Kolmogorov
    c = W.learned_holdout()[0]
    op = Kolmogorov.kolmogorov(N, c["alpha"], c["Re"], c["dt"], c["T"], c["n_forcing"])
    w = op.project(W.kolmo_start_physical(N, 0))
    t0 = time.perf_counter()
    count = 0
    while True:
        w = op.apply(w)
        w /= np.linalg.norm(w)
        count += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    ms_mv = el * 1e3 / count
    model, ncpu = cpu_model()
    return {"value": ms_mv * mean_matvecs, "unit": "ms per solve", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_logical_cores": ncpu,
            "ms_per_matvec": ms_mv,
            "sample": f"{count} oracle matvecs (200 IF-RK4 steps each) of the held-out {N}x{N} FP64 operator "
                      f"(Re={c['Re']:.3f}, alpha={c['alpha']}) in {el:.1f} s, NumPy/pocketfft single thread; "
                      f"value = ms per matvec x {mean_matvecs:.1f} (the FP64 form's mean matvecs per solve)"}


def _nearest_dist(vals, ref):
    """Largest distance from a value of `vals` to the nearest value of `ref`."""
    ref = np.asarray(ref)
    return max((float(np.min(np.abs(ref - v))) for v in vals), default=0.0)


def _true_residuals(tsk, torch, op64, r):
    """||M x - mu x|| of each unit Ritz vector under the FP64 operator (one FP64
    matvec of its real and one of its imaginary part)."""
    out = []
    for mu, x in zip(r["mu"], r["X"]):
        x = x / torch.linalg.norm(x)
        y = torch.zeros_like(x)
        for part, sc in ((x.real, 1.0), (x.imag, 1j)):
            a = part.contiguous().double()
            b = torch.zeros_like(a)
            tsk.apply(op64, a, b)
            y = y + sc * b
        out.append(float(torch.linalg.norm(y - complex(mu) * x)))
    return out


def run_sweep_tsgp(tsk, W, torch, reps=3):
    """Throughput of the 64-instance FP32 neutral-curve sweep (m = 64, k = 4):
    time-steps x gridpoints of the matvecs per second of whole-batch wall time."""
    sweep = W.batch_sweep(64, 0)
    ops = []
    for c in sweep:
        op = tsk.create_kolmo2d(c["N"], tsk.TSK_FP32)
        tsk.set_params_kolmo(op, c["Re"], c["alpha"], c["dt"], c["T"])
        tsk.set_base_kolmogorov(op, c["n_forcing"])
        ops.append(op)
    tsk.batch_krylov_schur(ops, 64, 4, 1e-8, delta=0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        rb = tsk.batch_krylov_schur(ops, 64, 4, 1e-8, delta=0.1)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    nsteps = int(round(sweep[0]["T"] / sweep[0]["dt"]))
    tsgp = sum(b["n_matvec"] * nsteps * c["N"] ** 2 for b, c in zip(rb, sweep))
    return {"tsgp_per_s": tsgp / el, "ms_per_sweep": el * 1e3,
            "converged": sum(b["status"] == tsk.TSK_OK for b in rb), "instances": len(rb),
            "restarted": sum(b["n_restarts"] > 0 for b in rb),
            "workload": "64 Kolmogorov instances (24x128^2, 20x256^2, 20x384^2), FP32, Re~U[5,40], "
                        "alpha in {0.25,0.5,0.75,1}, m=64, k=4, tol=1e-8, batched Krylov-Schur (delta 0.1, "
                        "p_max 32) for the instances not converged at order 64, one batched call"}


def run_learned(args, tsk, W, np, torch):
    """Headline: wall time to 6 Ritz pairs on held-out (Re, alpha) at 256^2, FP32
    + learned start against the plain FP64 + random start.  One solve = one
    tsk_arnoldi call from the start vector (the learned one includes the
    network's forward pass and decode) to the Ritz values and vectors; 16
    held-out instances, each solved once per step.  The network is trained
    first, outside the timed region, on Ritz vectors of the 64-instance sweep.

    Forms (all m = 96, k = 6, tol = 1e-8 on the Arnoldi residual estimate):
      fp64_random          the plain form (FP64 stop rule).
      fp32_learned         FP32 precision form, learned start; FP32 stop rule
                           (estimate <= max(1e-8, 1.9e-6 |mu|), duplicate width 2e-5).
      fp32_random          FP32 precision form, seeded random start.
      fp64_random_fp32rule FP64 + random start stopped by the FP32 rule: the
                           plain form at the precision form's accuracy.
    Accuracy (untimed, once per instance): the true residual ||M x - mu x|| of
    every returned pair by one FP64 matvec, and |dlambda| of every returned
    value to the nearest value of an FP64 run with k = 12."""
    floor = 32 * 2.0 ** -24
    t_train0 = time.perf_counter()
    sweep = W.learned_training_sweep()

    def mk(c, prec):
        op = tsk.create_kolmo2d(c["N"], prec)
        tsk.set_params_kolmo(op, c["Re"], c["alpha"], c["dt"], c["T"])
        tsk.set_base_kolmogorov(op, c["n_forcing"])
        return op

    sops = [mk(c, tsk.TSK_FP32) for c in sweep]
    res = tsk.batch_arnoldi(sops, sweep[0]["m"], sweep[0]["k"], sweep[0]["tol"], want_vectors=True)
    T = torch.stack([tsk.ritz_block_target(op, r["X"], [r["res"][i] <= max(c["tol"], floor * abs(r["mu"][i]))
                                                         for i in range(r["n_ritz"])])
                     for c, op, r in zip(sweep, sops, res)]).contiguous()
    x = torch.tensor([[c["Re"], c["alpha"]] for c in sweep], dtype=torch.float32, device="cuda")
    net = tsk.mlp_create(512, W.LEARNED_IN_LO, W.LEARNED_IN_HI)
    tsk.mlp_init(net, 0)
    losses = tsk.mlp_train(net, x, T, 3000, 1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train0
    del sops, res

    hold = W.learned_holdout()
    N = hold[0]["N"]
    m, k, tol = hold[0]["m"], hold[0]["k"], hold[0]["tol"]
    o64 = [mk(c, tsk.TSK_FP64) for c in hold]
    o64r = [mk(c, tsk.TSK_FP64) for c in hold]
    for op in o64r:
        tsk.set_stop_rule(op, floor, 2e-5)
    o32 = [mk(c, tsk.TSK_FP32) for c in hold]

    def p64(i, s):
        return tsk.arnoldi(o64[i], m, k, tol, seed=s, want_vectors=True)

    def p64r(i, s):
        return tsk.arnoldi(o64r[i], m, k, tol, seed=s, want_vectors=True)

    def p32r(i, s):
        return tsk.arnoldi(o32[i], m, k, tol, seed=s, want_vectors=True)

    def p32l(i, s):
        v0, _ = tsk.mlp_start(net, o32[i], hold[i]["Re"], hold[i]["alpha"], 0.1, s)
        return tsk.arnoldi(o32[i], m, k, tol, v0=v0, want_vectors=True)

    forms = {"fp64_random": p64, "fp32_learned": p32l, "fp32_random": p32r, "fp64_random_fp32rule": p64r}
    rules = {"fp64_random": "estimate <= 1e-8", "fp32_learned": "estimate <= max(1e-8, 1.9e-6|mu|), dup 2e-5",
             "fp32_random": "estimate <= max(1e-8, 1.9e-6|mu|), dup 2e-5",
             "fp64_random_fp32rule": "estimate <= max(1e-8, 1.9e-6|mu|), dup 2e-5"}
    # FP64 reference spectra (k = 12) for |dlambda|
    refs = [tsk.arnoldi(o64[i], m, 12, tol, seed=7)["lam"] for i in range(len(hold))]
    stats, last = {}, {}
    for name, fn in forms.items():
        for w in range(args.warmup):
            for i in range(len(hold)):
                fn(i, 1000 + w * 100 + i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nmv, nok, ms_apply = [], 0, 0.0
        for st in range(args.steps):
            for i in range(len(hold)):
                r = fn(i, st * 100 + i)
                nmv.append(r["n_matvec"])
                nok += r["status"] == tsk.TSK_OK
                ms_apply += r["ms_apply"]
                last[(name, i)] = r
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        nsolve = args.steps * len(hold)
        stats[name] = {"ms_per_solve": el * 1e3 / nsolve, "mean_matvecs": float(np.mean(nmv)),
                       "converged": nok, "solves": nsolve, "stop_rule": rules[name],
                       "matvec_ms_per_solve": ms_apply / nsolve,
                       "ms_per_matvec": ms_apply / float(np.sum(nmv))}
        print(name, stats[name], file=sys.stderr)
    for name in forms:
        tr, dl, est = [], [], []
        for i in range(len(hold)):
            r = last[(name, i)]
            tr += _true_residuals(tsk, torch, o64[i], r)
            dl.append(_nearest_dist(r["lam"], refs[i]))
            est += list(r["res"])
        stats[name].update({"max_true_residual": max(tr), "median_true_residual": float(np.median(tr)),
                            "max_estimate": float(max(est)), "max_dlambda_vs_fp64": max(dl),
                            "median_dlambda_vs_fp64": float(np.median(dl))})
    lm = stats["fp32_learned"]["ms_per_solve"]
    nsteps = int(round(hold[0]["T"] / hold[0]["dt"]))
    launch_ms = stats["fp32_learned"]["ms_per_matvec"]
    flops, kname = stepper_flops(tsk, o32[0], N, nsteps)
    achieved = flops / (launch_ms / 1e3) / 1e12
    traffic = measured_traffic("k_colstep_couple_kolmo256_fp32_hbm_traffic.md",
                               key=f"traffic_bytes_per_launch_w{tsk.get_stepper_waves(o32[0])}")
    sweep_stats = run_sweep_tsgp(tsk, W, torch)
    for name in forms:
        stats[name]["tsgp_per_s"] = stats[name]["mean_matvecs"] * nsteps * N * N / (stats[name]["ms_per_solve"] / 1e3)
    return {
        "metric": "wall time to 6 Ritz pairs (Arnoldi estimate <= 1e-8; FP32 form: its precision floor) "
                  "on held-out 256^2 instances, FP32 + learned start vs plain FP64 + random start",
        "value": lm, "unit": "ms per solve", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": lm * len(hold), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "16 held-out (Re~U[5,40] seed 1000, alpha in {0.25,0.5,0.75,1}) linearized "
                               "Kolmogorov flows 256x256, IF-RK4 dt=0.005 T=1, Arnoldi m=96 k=6 tol=1e-8, "
                               "Ritz vectors returned; FP32 + learned start (gamma 0.1) vs FP64 + seeded random "
                               "start; a step = one solve of each of the 16 instances",
                   "forms": stats,
                   "speedup_vs_fp64_random": stats["fp64_random"]["ms_per_solve"] / lm,
                   "speedup_vs_fp64_random_at_fp32_rule": stats["fp64_random_fp32rule"]["ms_per_solve"] / lm,
                   "time_steps_x_gridpoints_per_s": stats["fp32_learned"]["tsgp_per_s"],
                   "sweep": sweep_stats,
                   "training": {"instances": len(sweep), "adam_steps": 3000, "lr": 1e-3,
                                "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                                "sweep_and_train_s": t_train}},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "launch_ms": launch_ms, "flops_per_launch": flops, "traffic": traffic},
        "cpu_baseline": None if args.no_cpu_baseline else
        cpu_baseline_learned(N, stats["fp64_random"]["mean_matvecs"]),
    }


def cn_pcr_flops(n, levels):
    """Flops of one Crank-Nicolson step of the cyclic-reduction kernel per node:
    the three-point explicit half (3 complex multiplies, 2 adds: 22), the forcing
    term (8), per reduction level two complex multiply-adds (16) and the final
    scaling (6)."""
    return n * (22 + 8 + 16 * levels + 6)


def cpu_baseline_cgle(c, seconds=10.0):
    """The CPU oracle's Crank-Nicolson matvecs (banded solve per step, single
    thread) of the same Ginzburg-Landau operator, as many as fit in `seconds`."""
    import workloads as W
    from oracle.cgle import CGLE
    op = CGLE(n=c["n"], half_width=c["half_width"], U=c["U"], c_u=c["c_u"], c_d=c["c_d"], mu0=c["mu0"],
              mu2=c["mu2"], dt=c["dt"], T=c["T"])
    u = W.cgle_start(c["n"], 0)
    t0 = time.perf_counter()
    count = 0
    while True:
        u = op.apply(u)
        u /= np.linalg.norm(u)
        count += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    nsteps = int(round(c["T"] / c["dt"]))
    model, ncpu = cpu_model()
    return {"value": count * nsteps * c["n"] / el, "unit": "time-steps*gridpoints/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_logical_cores": ncpu,
            "sample": f"{count} oracle matvecs ({nsteps} Crank-Nicolson steps each) of the n={c['n']} operator, "
                      f"{el:.1f} s, NumPy/SciPy single thread"}


def run_cgle(args, tsk, W, np, torch):
    """Ginzburg-Landau (Sec. 2.3.2 operator; n = 256 finite-difference nodes on
    [-50, 50], Crank-Nicolson dt = 0.01, T = 1): Arnoldi m = 64, k = 6, tol =
    1e-8 from the seeded complex N(0,1) start.  A step is one whole run."""
    c = W.CGLE
    n, m, k, tol = c["n"], c["m"], c["k"], c["tol"]
    nsteps = int(round(c["T"] / c["dt"]))
    op = tsk.create_cgle1d(n, c["half_width"])
    tsk.set_params_cgle(op, c["U"], c["c_u"], c["c_d"], c["mu0"], c["mu2"], c["dt"], c["T"])
    v0 = torch.from_numpy(W.cgle_start(n, 0)).cuda()

    def step():
        return tsk.arnoldi(op, m, k, tol, v0=v0, want_vectors=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    r = results[-1]
    nmv = r["n_matvec"]
    ms_apply = sum(q["ms_apply"] for q in results) / args.steps
    launch_ms = ms_apply / nmv
    levels = int(math.ceil(math.log2(n)))
    flops = nsteps * cn_pcr_flops(n, levels)
    achieved = flops / (launch_ms / 1e3) / 1e12
    tsgp = nmv * nsteps * n
    return {
        "metric": "time-steps*gridpoints/s (whole Arnoldi run to 6 Ritz pairs at residual 1e-8)",
        "value": tsgp / (ms / 1e3), "unit": "time-steps*gridpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"linear complex Ginzburg-Landau n={n} finite-difference nodes on [-50,50], U=2, "
                               f"c_u=0.2, c_d=-1, mu0=0.41, mu2=-0.01, Crank-Nicolson dt={c['dt']} T={c['T']}, "
                               f"Arnoldi m={m} k={k} tol={tol}, seeded complex N(0,1) start",
                   "n_matvec": nmv, "status": r["status"], "us_per_cn_step": launch_ms * 1e3 / nsteps,
                   "time_stepper_tsgp_per_s": tsgp / (ms_apply / 1e3),
                   "lambda": [[round(float(v.real), 10), round(float(v.imag), 10)] for v in r["lam"]],
                   "max_residual": float(np.max(r["res"]))},
        "roofline": {"bound": "alu", "kernel": f"k_cgle_cn<{levels}> (one workgroup, latency-bound)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "launch_ms": launch_ms,
                     "flops_per_launch": flops, "traffic": None},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_cgle(c),
    }


def cpu_baseline_resolvent(n, half_width, mu0, dt, t_trans, omega, seconds=10.0):
    """The CPU oracle's forced integration (banded LAPACK solve per step, single
    thread) of the same resolvent operator: as many whole integrations as fit in
    about `seconds`."""
    import numpy as np

    import workloads as W
    from oracle.cgle import CGLE
    from oracle.resolvent import forced_response
    op = CGLE(n=n, half_width=half_width, mu0=mu0, dt=dt)
    f = W.normal_complex(n, 0)
    t0 = time.perf_counter()
    count = 0
    while True:
        f = forced_response(op, f, omega, t_trans, adjoint=bool(count % 2))
        f /= np.linalg.norm(f)
        count += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    nsteps = int(round(t_trans / dt))
    return {"value": count * nsteps * n / el, "unit": "time-steps*gridpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"{count} oracle forced integrations (R and R^H alternately, {nsteps} Crank-Nicolson steps "
                      f"each) of the n={n} operator at omega={omega}, {el:.1f} s, NumPy/SciPy single thread"}


def run_resolvent(args, tsk, W, np, torch):
    """Resolvent analysis of the linear complex Ginzburg-Landau equation (Sec.
    2.3.2 illustration: mu0 = 0.23, x in [-85, 85]; Sec. 3.3.2 forced time
    integration): the first four gains sigma_j^2 at 64 forcing frequencies in
    [-1.5, 0.5].  Each frequency is one operator in resolvent mode (23000
    Crank-Nicolson steps from rest, dt = 0.01, t = 230); Lanczos on R^H R to
    residual 1e-6 for all 64 in one batch (one workgroup per frequency).  A step
    is the whole sweep from seeded starts."""
    n, hw, mu0, dt, tt = 400, 85.0, 0.23, 0.01, 230.0
    F, m, k, tol = 64, 48, 4, 1e-6
    omegas = np.linspace(-1.5, 0.5, F)
    ops = []
    for w in omegas:
        op = tsk.create_cgle1d(n, hw)
        tsk.set_params_cgle(op, 2.0, 0.2, -1.0, mu0, -0.01, dt, 1.0)
        tsk.set_resolvent(op, float(w), tt)
        ops.append(op)
    seeds = list(range(F))

    def run():
        return tsk.batch_optimal_perturbation(ops, m, k, tol, seeds=seeds)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [run() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = el * 1e3 / args.steps
    r = results[-1]
    nsteps = int(round(tt / dt))
    levels = int(math.ceil(math.log2(n)))
    steps = [q["n_steps"] for q in r]
    lockstep = max(steps)
    useful = sum(2 * q * nsteps * n for q in steps)  # forward + adjoint per Lanczos step
    ms_apply = sum(q[0]["ms_apply"] for q in results) / args.steps
    launch_ms = ms_apply / (2 * lockstep)
    flops = F * nsteps * cn_pcr_flops(n, levels)
    achieved = flops / (launch_ms / 1e3) / 1e12
    gains = np.array([q["gain"] for q in r])
    ipk = int(np.argmax(gains[:, 0]))
    return {
        "metric": "time-steps*gridpoints/s (resolvent gain sweep: 64 frequencies, 4 gains each, Lanczos on R^H R "
                  "at residual 1e-6, R by forced time integration)",
        "value": useful / (ms_per_step / 1e3),
        "unit": "time-steps*gridpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"resolvent of the linear complex Ginzburg-Landau equation, n={n} finite-difference "
                               f"nodes on [-85,85], U=2, c_u=0.2, c_d=-1, mu0=0.23, mu2=-0.01, Crank-Nicolson "
                               f"dt={dt}, forced from rest over t={tt}; {F} frequencies in [-1.5,0.5]; Lanczos "
                               f"m={m} k={k} tol={tol}, seeded N(0,1) starts",
                   "lanczos_steps": steps, "status": [q["status"] for q in r],
                   "omega": [float(w) for w in omegas], "gains": gains.tolist(),
                   "peak": {"omega": float(omegas[ipk]), "gain": float(gains[ipk, 0])},
                   "lockstep_integrations": 2 * lockstep,
                   "time_stepper_tsgp_per_s": F * nsteps * n / (launch_ms / 1e3)},
        "roofline": {"bound": "alu", "kernel": "k_cgle_cn_batch (64 workgroups, one per frequency)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "launch_ms": launch_ms,
                     "flops_per_launch": flops, "traffic": None},
        "cpu_baseline": None if args.no_cpu_baseline else
        cpu_baseline_resolvent(n, hw, mu0, dt, tt, float(omegas[ipk])),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="learned",
                    choices=["learned", "kolmo128", "kolmo256-fp32", "kolmo512-fp32", "sweep", "cgle", "general", "krylov-schur",
                             "optimal", "fixed-point", "resolvent", "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1804_03859_amd.tsk as tsk
    import workloads as W

    if not os.path.exists(tsk.LIB_PATH):
        from paper_1804_03859_amd import build
        build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "kolmo128":
        out = run_single(args, tsk, W, np, torch, W.KOLMO_128_FP64, tsk.TSK_FP64, "f64")
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline()
    elif args.workload == "copy":
        # calibration of the HBM byte counters: plain device copies of a known size
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out = {"metric": "copy calibration", "value": 2 * nbytes * args.steps / el / 1e9, "unit": "GB/s",
               "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes, "steps": args.steps}
    elif args.workload == "kolmo256-fp32":
        out = run_single(args, tsk, W, np, torch, dict(W.KOLMO_512_FP32, N=256), tsk.TSK_FP32, "f32")
    elif args.workload == "kolmo512-fp32":
        out = run_single(args, tsk, W, np, torch, W.KOLMO_512_FP32, tsk.TSK_FP32, "f32")
    elif args.workload == "learned":
        out = run_learned(args, tsk, W, np, torch)
    elif args.workload == "general":
        out = run_general(args, tsk, W, np, torch)
    elif args.workload == "cgle":
        out = run_cgle(args, tsk, W, np, torch)
    elif args.workload == "krylov-schur":
        out = run_krylov_schur(args, tsk, W, np, torch)
    elif args.workload == "optimal":
        out = run_optimal(args, tsk, W, np, torch)
    elif args.workload == "fixed-point":
        out = run_fixed_point(args, tsk, W, np, torch)
    elif args.workload == "resolvent":
        out = run_resolvent(args, tsk, W, np, torch)
    else:
        out = run_sweep(args, tsk, W, np, torch)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
