"""Benchmark: CPR-GMRES solves/s on the 4M-cell (200x200x100) 4x4-block system,
FP32-stored preconditioner inside FP64 GMRES (headline) beside plain FP64,
plus the HBM roofline of the block SpMV and the FP64 CPU oracle's rate.

One step = one Newton-step linear solve on the whole path: take the new
values in place and decouple them (ABF) in one pass (rs_bsr_attach_decouple:
the Jacobian stays in the caller's device buffer, no copy), CPR setup
(AMG + layer RAS), and restarted GMRES from x0 = 0 to a true FP64 relative
residual of 1e-8.  Inputs are seeded synthetic draws already resident in HBM;
the Jacobian is assembled on the device.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# second stage: zero-overlap RAS over xy-layers with DILU inside (default),
# RAS with overlap 1, DILU of the whole matrix, or block Jacobi
SMOOTHERS = {"bj": 0, "dilu": 1, "ras": 2, "ras1": 3}
DECOUPLINGS = {"abf": 0, "qi": 1, "frs": 2, "frs_abf": 3}
SMOOTHER_NAMES = {"bj": "block Jacobi", "dilu": "DILU", "ras": "RAS(0, xy-layers) + DILU",
                  "ras1": "RAS(1, xy-layers) + DILU"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def spmv_roofline(rs, A, n, reps=20):
    import torch
    N = 4 * n
    x = torch.randn(N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        rs.spmv(A, x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        rs.spmv(A, x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # algorithmic bytes of one y = A x: stored blocks (128 B each) + x + y;
    # the structured layout reads no index arrays
    nbytes = A.nnzb * 128 + 2 * N * 8
    return ms, nbytes


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv7_cfg2_traffic.txt")
SPMV_SOURCE = os.path.join(ROOT, "paper_1812_03952_amd", "csrc", "bsr.hip")


def spmv_traffic(cells):
    """HBM bytes per SpMV launch from the committed counter summary, or None
    when the SpMV source has changed since the counters were taken or the
    counters were taken on a grid of another size."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        cur = hashlib.sha256(open(SPMV_SOURCE, "rb").read()).hexdigest()
        if kv.get("source_sha256") != cur or int(kv.get("cells", -1)) != cells:
            return None
        return float(kv["traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def calibration_copy():
    """A plain copy of exactly 1 GiB (read) into 1 GiB (write), outside every
    timed region: under rocprofv3 --pmc its FETCH_SIZE/WRITE_SIZE give the
    scale between the counters and bytes."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def run_variant(rs, dp, A, prec, steps, warmup, tag, smoother, solver="gmres", method=0, stages=2, smooth=0):
    import torch
    times, infos, phases = [], [], []
    for it in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        D = rs.bsr_attach_decouple(A, dp.vals, method, prec)   # new Jacobian values, decoupled
        t1 = time.perf_counter()
        M = rs.cpr_setup(A, D, rs.cpr_opts(smoother=smoother, stages=stages, smooth=smooth))
        t2 = time.perf_counter()
        # x0 = 0 by zero_guess: the solvers take r0 = b without a product with
        # A and never read x before writing it
        x = torch.empty_like(dp.b)
        if solver == "gmres":
            info = rs.gmres_solve(A, M, dp.b, x, rs.gmres_opts(zero_guess=1))
        else:
            info = rs.bicgstab_solve(A, M, dp.b, x, rs.bicgstab_opts(zero_guess=1))
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        del M, D
        if it >= warmup:
            times.append(t3 - t0)
            infos.append(info)
            phases.append((t1 - t0, t2 - t1, t3 - t2))
        log(f"[{tag}] step {it} ({'warmup' if it < warmup else 'timed'}): {1e3 * (t3 - t0):.1f} ms "
            f"iters={info['iters']} relres={info['relres']:.2e}")
    return times, infos, phases


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    return model, ncores


def cpu_baseline(prob, smoother):
    import oracle
    t0 = time.perf_counter()
    A = oracle.assemble(prob)
    t1 = time.perf_counter()
    M = oracle.CPR(A, smoother=smoother)
    x, info = oracle.gmres(A, prob.b, M, rtol=1e-8)
    t2 = time.perf_counter()
    return t2 - t1, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--solvers", default="gmres,bicgstab",
                    help="comma list of outer solvers, each run with the FP32 preconditioner; the first is the "
                         "headline (the FP64 variant runs with GMRES when gmres is listed)")
    ap.add_argument("--smoother", choices=list(SMOOTHERS), default="ras")
    ap.add_argument("--decouple", choices=list(DECOUPLINGS), default="abf")
    ap.add_argument("--stages", type=int, choices=[2, 3], default=2,
                    help="CPR stages: 2 = pressure then full, 3 = CPR-FPF")
    ap.add_argument("--amg", choices=["ua", "sa"], default="ua",
                    help="pressure AMG prolongator: piecewise constant (ua) or smoothed and truncated (sa)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB copy kernel (for counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1812_03952_amd import rsolve as rs

    torch.cuda.set_device(0)
    if args.calib_copy:
        calibration_copy()
    t = time.perf_counter()
    prob = synth.config(args.config)
    log(f"draws for {prob.name}: {time.perf_counter() - t:.1f} s")
    dp = rs.DeviceProblem(prob)
    torch.cuda.synchronize()
    A = dp.bsr()
    n = prob.n

    res = {}
    solvers = [x for x in args.solvers.split(",") if x]
    if not solvers or any(x not in ("gmres", "bicgstab") for x in solvers):
        sys.exit("bench.py: --solvers takes gmres and/or bicgstab")
    variants = []
    for sv in solvers:
        variants.append(("fp32" if sv == "gmres" else "bicgstab_fp32", 32, sv))
        if sv == "gmres" and not args.no_fp64:
            variants.append(("fp64", 64, "gmres"))
    for tag, prec, solver in variants:
        times, infos, phases = run_variant(rs, dp, A, prec, args.steps, args.warmup, tag, SMOOTHERS[args.smoother],
                                           solver, DECOUPLINGS[args.decouple], args.stages,
                                           1 if args.amg == "sa" else 0)
        tmax = max(times)
        tmed = float(np.median(times))
        ph = np.median(np.array(phases), axis=0)
        res[tag] = dict(solves_per_s=len(times) / sum(times), ms_per_solve=1e3 * tmed, ms_max=1e3 * tmax,
                        iters=infos[-1]["iters"], relres=infos[-1]["relres"],
                        ms_decouple=1e3 * ph[0], ms_cpr_setup=1e3 * ph[1], ms_krylov=1e3 * ph[2], solver=solver,
                        solve_only_per_s=1.0 / ph[2])
    spmv_ms, spmv_bytes = spmv_roofline(rs, A, n)
    achieved = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    head = res[variants[0][0]]
    steps_total = sum(1 for _ in range(args.steps))
    out = {
        "metric": "CPR-GMRES solves/s + SpMV HBM GB/s at 4M cells; FP32-precond vs FP64",
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps_total,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-preconditioner/fp64-gmres",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: 4x4-block 7-point Jacobian, {n} cells, {4 * n} unknowns, "
                               f"nnzb {A.nnzb}; {args.decouple.upper()} + {'CPR-FPF' if args.stages == 3 else 'CPR'}({'smoothed-aggregation ' if args.amg == 'sa' else ''}AMG V-cycle, "
                               f"{SMOOTHER_NAMES[args.smoother]}) + {'FGMRES(30)' if solvers[0] == 'gmres' else 'BiCGSTAB'}, rtol 1e-8",
                   "cells": n, "unknowns": 4 * n, "nnzb": A.nnzb, "restart": 30, "rtol": 1e-8,
                   "smoother": args.smoother, "headline_solver": solvers[0], "decouple": args.decouple,
                   "cpr_stages": args.stages, "amg": args.amg},
        "fp32_precond": res.get("fp32"),
        "fp64": res.get("fp64"),
        "bicgstab_fp32_precond": res.get("bicgstab_fp32"),
        "spmv": {"ms": spmv_ms, "GB_per_s": achieved, "bytes": spmv_bytes},
        "roofline": {"bound": "hbm", "kernel": "k_spmv7<double,false,0,true> (y = A x, values read in place)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": spmv_traffic(n)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle, one full solve of the same system (1 thread) ...")
        t_cpu, info = cpu_baseline(prob, SMOOTHERS[args.smoother])
        model, ncores = host_cpu()
        # the oracle is single-threaded C: its sweeps, the greedy MIS and the
        # GMRES reductions are sequential by definition, so it uses one core
        out["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "host_cores": ncores, "cpu_model": model,
                               "sample": f"one complete FP64 CPR-GMRES solve of {prob.name} (decouple, AMG and "
                                         f"{args.smoother} set-up, GMRES to 1e-8: {info['iters']} iterations) on one "
                                         f"of the host's {ncores} cores, {t_cpu:.1f} s; the assembly is not timed"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
