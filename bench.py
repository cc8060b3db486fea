#!/usr/bin/env python3
"""Coupled-update throughput of the electrofreezing lattice Boltzmann hot path on one MI355X.

A step is one full time step of Algorithm 1 on the 1024 x 512 sessile-drop workload (f, the
potential swept to a relative change of 1e-8, h, g and every coupling term), all in the HIP
library; inputs are resident in HBM before the timed region.  Prints one JSON line with the
coupled MLUPS, the roofline of the dominant kernel (the potential sweep) and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled MLUPS + % HBM roofline; time-to-freeze, plain FP64 vs FP32/batched/warm"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
SWEEP_BYTES_FP64 = 88  # per node: 4 links + phi + 1/tau_l read, 4 links + phi written


def workload(name):
    from paper_2410_06657_amd import inputs
    if name == "cfg2":
        c = inputs.cfg2(90.0, "prolate", 0.1)
        desc = "1024x512 sessile drop, R0=160, theta=90, R=3, S=1 (prolate), Ca_E=0.1, Ste=0.1, rho_l/rho_g=10, k_s/k_l=2"
    elif name == "cfg1":
        c = inputs.cfg1(0)
        desc = "128x64 sessile drop, R0=24, theta=90, R=3, S=1, Ca_E=0.1, Ste=0.1, seed 0"
    elif name == "cfg3":
        c = inputs.cfg3()
        desc = "4096x2048 sessile drop, R0=640, theta=90, R=3, S=1, Ca_E=0.1, Ste=0.1"
    else:
        raise SystemExit(f"unknown workload {name}")
    return c, desc


def cpu_baseline(case, k_sweeps, budget_s=25.0):
    """Oracle on the host cores: per-sweep time and the rest of a step, measured on the same
    grid, combined into one coupled step with the GPU's mean sweep count."""
    from oracle.binding import Oracle, set_threads
    threads = os.cpu_count() or 1
    set_threads(threads)
    c = dict(case, poisson_tol=-1.0, poisson_max_sweeps=2)
    o = Oracle(c)  # fields, equilibria and a 2-sweep potential solve
    t0 = time.perf_counter()
    o.solve_potential(-1.0, 5)
    per_sweep = (time.perf_counter() - t0) / 5
    nsw = max(5, min(200, int(budget_s * 0.5 / max(per_sweep, 1e-9))))
    t0 = time.perf_counter()
    o.solve_potential(-1.0, nsw)
    per_sweep = (time.perf_counter() - t0) / nsw
    t0 = time.perf_counter()
    o.step(1)  # one step with two (fixed) sweeps
    rest = time.perf_counter() - t0 - 2 * per_sweep
    step_s = rest + k_sweeps * per_sweep
    n = case["nx"] * case["ny"]
    return {"value": n / step_s / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{case['nx']}x{case['ny']} grid: {nsw} timed oracle sweeps "
                      f"({per_sweep * 1e3:.2f} ms each) and one step with two sweeps "
                      f"({rest * 1e3:.1f} ms besides the sweep), combined as one step with "
                      f"{k_sweeps:.1f} sweeps (the GPU's mean)",
            "step_s": step_s}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--sweep-launches", type=int, default=200,
                    help="sweep launches timed with HIP events for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no "
              "multi-GPU path; see the sharding notes in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_06657_amd.lbm import Solver

    case, desc = workload(args.workload)
    n = case["nx"] * case["ny"]
    t0 = time.perf_counter()
    s = Solver(case)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    print(f"[bench] init {init_s:.1f}s, initial solve {s.sweep_log()[0]} sweeps", file=sys.stderr, flush=True)
    s.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)
    nlog = len(s.sweep_log())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweeps = s.sweep_log()[nlog:]
    kmean = float(np.mean(sweeps))
    ms_step = dt / args.steps * 1e3
    value = n * args.steps / dt / 1e6
    d = s.diag()
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step, {kmean:.1f} sweeps/step",
          file=sys.stderr, flush=True)

    # dominant kernel: the potential sweep, timed live with HIP events on the solver's stream
    ms = s.time_sweeps(args.sweep_launches)
    avg_s = ms * 1e-3 / args.sweep_launches
    per_launch = SWEEP_BYTES_FP64 * n
    achieved = per_launch / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_sweep", "avg_us": round(avg_s * 1e6, 3),
                "algorithmic_bytes_per_launch": per_launch}

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "nx": case["nx"], "ny": case["ny"], "precision": "fp64",
                   "poisson_tol": case["poisson_tol"]},
        "sweeps_per_step": round(kmean, 2),
        "sweep_time_share": round(min(1.0, kmean * avg_s * 1e3 / ms_step), 4),
        "init_s": round(init_s, 2),
        "roofline": roofline,
        "state": {"step": d["step"], "V_s": d["V_s"], "height": d["height"], "nonfinite": d["nonfinite"]},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(case, kmean)
        cb.pop("step_s")
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
