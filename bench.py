#!/usr/bin/env python3
"""Coupled-update throughput of the electrofreezing lattice Boltzmann hot path on one MI355X.

A step is one full time step of Algorithm 1 on the 4096 x 2048 sessile-drop workload (f, the
potential swept to a relative change of 1e-8, h, g and every coupling term), all in the HIP
library; inputs are resident in HBM before the timed region.  The initial potential is seeded
by the learned warm start and swept to the same stopping rule before anything is timed (the
run fails if that solve reaches its cap).  Each form runs with the launch shapes the library's
autotuner picks for it.  Prints one JSON line with the coupled MLUPS, the roofline of the kernel
that takes the most time per step, the rooflines of every kernel of the step, a plain copy's HBM
rate beside the peak, the precision forms at the same size, and the CPU oracle timed on a
bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled MLUPS + % HBM roofline; time-to-freeze, plain FP64 vs FP32/batched/warm"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
INFINITY_CACHE_BYTES = 256 << 20  # MI355X last-level (Infinity) cache in front of HBM
# algorithmic bytes per node (element size s): a potential sweep reads 4 links, phi and
# 1/tau_l and writes 4 links and phi (11 s); a step outside the sweeps moves 27 + 27
# populations and 13 + 13 fields (80 s)
SWEEP_ELEMS, STEP_ELEMS = 11, 80
ELEM = {"fp64": 8, "fp32": 4, "fp16store": 4}
# bytes per node of a step outside the sweeps; the FP16-storage form moves its 54 populations
# as binary16 and its 26 field values as floats
STEP_BYTES = {"fp64": STEP_ELEMS * 8, "fp32": STEP_ELEMS * 4, "fp16store": 54 * 2 + 26 * 4}
# compulsory HBM bytes per node of one blocked sweep launch (read once, written once, whatever
# the number of sweeps): FP64 reads 4 links and 1/tau_l and writes 4 links and phi; FP32 reads
# 4 link remainders, 1/tau_l, the 4 pulled base increments and phi_B and writes 4 remainders
# and phi
SWEEP_COMPULSORY = {"fp64": 10 * 8, "fp32": 15 * 4, "fp16store": 15 * 4}
# bytes per node each kernel of the step must read and write when every neighbour it uses is
# served on chip (populations 8 / 4 / 2 B, fields 8 / 4 / 4 B):
#   f: f 9 + 9; psi, u (2), (psi u)^{n-1} (2), mdot, f_s in; psi, 1/tau_l out
#   h: h 9 + 9; psi^{n+1}, f_s, phi, p, u (2), u* (2), mdot in; p, u (2), u* (2) out (every
#     coupling term of the flow step is evaluated on chip)
#   g: g 9 + 9; H, T, psi (2 levels), f_s, u (2 levels x 2), mdot in; H, T, f_s, mdot, f_l,
#     (psi u) (2) out; the FP32 forms also read and write the enthalpy base
KERNEL_BYTES = {
    "k_f_fused_arm": {"fp64": 27 * 8, "fp32": 27 * 4, "fp16store": 18 * 2 + 9 * 4},
    "k_h_fused": {"fp64": 32 * 8, "fp32": 32 * 4, "fp16store": 18 * 2 + 14 * 4},
    "k_g_stream": {"fp64": 35 * 8, "fp32": 37 * 4, "fp16store": 18 * 2 + 19 * 4},
}

COUNTERS_FILE = os.path.join(ROOT, "profiles", "kernels_4096x2048_counters.md")
BATCH_STAGE_ROWS = 32
KERNEL_SOURCE = os.path.join(ROOT, "paper_2410_06657_amd", "csrc", "lbm_kernels.hpp")


def kernel_source_digest():
    """SHA-256 of the kernel source and the compiler flags the counters must have been taken
    with (a flag such as -ffp-contract changes the code without touching the source)."""
    from paper_2410_06657_amd.build import HIPFLAGS
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read() + "\n".join(HIPFLAGS).encode()).hexdigest()


def measured_traffic(kernel, precision, workload_name, shapes=None):
    """HBM bytes per launch of a kernel from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE passes scaled by a copy kernel's), or None when the summary is missing, covers
    another workload, was taken from a different kernel source or with other launch shapes
    (sweep block, sweep waves, stage rows)."""
    if workload_name != "4096x2048" or not os.path.exists(COUNTERS_FILE):
        return None
    sha, table, taken = None, {}, {}
    with open(COUNTERS_FILE) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "kernel_source_sha256":
                sha = parts[1]
            elif len(parts) >= 4 and parts[0] == "traffic_bytes_per_launch":
                table[(parts[1], parts[2])] = int(parts[3])
            elif len(parts) == 5 and parts[0] == "launch_shapes":
                taken[parts[1]] = tuple(int(v) for v in parts[2:])
    if sha is None or sha != kernel_source_digest():
        return None
    if shapes is not None and taken.get(precision) != shape_key(shapes):
        return None
    return table.get((kernel, precision))


def shape_key(shapes):
    return (int(shapes["sweep_block"]), int(shapes["sweep_waves"]), int(shapes["stage_rows"]))


# the autotuner's timings by (nx, ny, precision), for the report
TUNE_TIMINGS = {}


def launch_shapes(case, precision, tune=True):
    """Launch shapes for a grid and precision: the library's autotuner (timed here, not taken
    from a file), or the library's defaults with tune=False."""
    if not tune:
        from paper_2410_06657_amd.lbm import launch_shapes as defaults
        return defaults(case, precision)
    from paper_2410_06657_amd.lbm import autotune
    r = autotune(dict(case, poisson_max_sweeps=2000), precision, launches=10, persist=False)
    TUNE_TIMINGS[(case["nx"], case["ny"], precision)] = {
        "us_per_sweep": {f"{k['sweep_block']}x{k['sweep_waves']}": round(k["us_per_sweep"], 3)
                         for k in r["candidates"]},
        "us_per_step_stages": {str(k["stage_rows"]): round(k["us_per_step"], 2) for k in r["stage_candidates"]}}
    return {"sweep_block": r["sweep_block"], "sweep_waves": r["sweep_waves"], "stage_rows": r["stage_rows"]}


def workload(name):
    from paper_2410_06657_amd import inputs
    if name == "4096x2048":
        c = inputs.drop_4096x2048()
        desc = "4096x2048 sessile drop, R0=640, theta=90, R=3, S=1 (prolate), Ca_E=0.1, Ste=0.1, rho_l/rho_g=10, k_s/k_l=2"
    elif name == "1024x512":
        c = inputs.drop_1024x512(90.0, "prolate", 0.1)
        desc = "1024x512 sessile drop, R0=160, theta=90, R=3, S=1 (prolate), Ca_E=0.1, Ste=0.1, rho_l/rho_g=10, k_s/k_l=2"
    elif name == "128x64":
        c = inputs.drop_128x64(0)
        desc = "128x64 sessile drop, R0=24, theta=90, R=3, S=1, Ca_E=0.1, Ste=0.1, seed 0"
    else:
        raise SystemExit(f"unknown workload {name}")
    return c, desc


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """HBM rate of a plain device-to-device copy of `nbytes` (2 x nbytes moved), `reps` copies
    timed with HIP events: the library's streaming copy kernel (lbm_time_copy, 16-byte loads
    and stores) and torch's copy.  What a streaming kernel reaches on this GPU, beside the
    8 TB/s peak the rooflines are quoted against."""
    import torch

    from paper_2410_06657_amd.lbm import time_copy
    lib_ms = time_copy(nbytes, reps)
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    torch_ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    rate = lambda ms: round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    return {"bytes_per_copy": 2 * nbytes, "achieved": rate(lib_ms), "unit": "GB/s",
            "frac_of_peak": round(rate(lib_ms) / HBM_PEAK_GBS, 4), "avg_copy_us": round(lib_ms * 1e3, 1),
            "kernel": "lbm_time_copy", "torch_copy_achieved": rate(torch_ms)}


def host_cpu():
    """The host's CPU model (first "model name" of /proc/cpuinfo) and the cores this process
    may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": usable}


def cpu_baseline(case, k_sweeps, budget_s=25.0):
    """Oracle on the host cores: per-sweep time and the rest of a step, measured on the same
    grid, combined into one coupled step with the GPU's mean sweep count."""
    from oracle.binding import Oracle, set_threads
    threads = host_cpu()["nproc"]
    set_threads(threads)
    c = dict(case, poisson_tol=-1.0, poisson_max_sweeps=2)
    o = Oracle(c)  # fields, equilibria and a 2-sweep potential solve
    t0 = time.perf_counter()
    o.solve_potential(-1.0, 3)
    per_sweep = (time.perf_counter() - t0) / 3
    nsw = max(3, min(200, int(budget_s * 0.4 / max(per_sweep, 1e-9))))
    t0 = time.perf_counter()
    o.solve_potential(-1.0, nsw)
    per_sweep = (time.perf_counter() - t0) / nsw
    t0 = time.perf_counter()
    o.step(1)  # one step with two (fixed) sweeps
    rest = time.perf_counter() - t0 - 2 * per_sweep
    step_s = rest + k_sweeps * per_sweep
    n = case["nx"] * case["ny"]
    return {"value": n / step_s / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sweeps_per_s": 1.0 / per_sweep, "host": host_cpu(),
            "sample": f"{case['nx']}x{case['ny']} grid: {nsw} timed oracle sweeps "
                      f"({per_sweep * 1e3:.2f} ms each) and one step with two sweeps "
                      f"({rest * 1e3:.1f} ms besides the sweeps), combined as one step with "
                      f"{k_sweeps:.1f} sweeps (the GPU's mean)",
            "step_s": step_s}


def roofline_of(kernel, precision, n, seconds, workload_name, bytes_per_node, sweeps=None, shapes=None):
    """HBM roofline of one kernel launch: algorithmic bytes over its live average duration."""
    per_launch = bytes_per_node * n
    achieved = per_launch / seconds / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4),
         "traffic": measured_traffic(kernel, precision, workload_name, shapes),
         "kernel": kernel, "avg_launch_us": round(seconds * 1e6, 2),
         "algorithmic_bytes_per_launch": per_launch,
         "working_set_fits_infinity_cache": per_launch <= INFINITY_CACHE_BYTES}
    if sweeps is not None:
        r["sweeps_per_launch"] = sweeps
    return r


def solver_converged(case, precision, net, factor, cap):
    """A solver whose initial potential is the network's seed swept to the stopping rule."""
    import torch

    from paper_2410_06657_amd.lbm import Solver
    t0 = time.perf_counter()
    s = Solver(dict(case, skip_initial_solve=1, poisson_max_sweeps=cap), precision)
    s.warm_start(net, factor)
    rc, k, r = s.solve_potential(case["poisson_tol"], cap)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if rc != 0:
        raise SystemExit(f"bench: the initial potential solve ({precision}) stopped at its cap of {cap} sweeps")
    print(f"[bench] {precision}: warm-started initial solve {k} sweeps, {dt:.1f} s", file=sys.stderr, flush=True)
    return s, k, dt


def run_form(case, precision, steps, warmup, sweep_launches, workload_name, net, factor, init_cap, tune=True):
    """Time `steps` coupled steps of one precision form from a converged potential, then each
    kernel of the step, with the launch shapes the autotuner picks for this precision."""
    import numpy as np
    import torch

    n = case["nx"] * case["ny"]
    shapes = launch_shapes(case, precision, tune)
    print(f"[bench] {precision}: launch shapes {shapes}", file=sys.stderr, flush=True)
    case = dict(case, **shapes)
    s, k_init, init_s = solver_converged(case, precision, net, factor, init_cap)
    s.step(warmup)
    torch.cuda.synchronize()
    nlog = len(s.sweep_log())
    noconv0 = s.diag()["noconv"]
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sweeps = s.sweep_log()[nlog:]
    kmean = float(np.mean(sweeps))
    ms_step = dt / steps * 1e3
    d = s.diag()
    capped = d["noconv"] - noconv0
    print(f"[bench] {precision}: {steps} steps, {ms_step:.3f} ms/step, {kmean:.1f} sweeps/step, "
          f"{capped} capped solves", file=sys.stderr, flush=True)
    fields = {k: s.field(k) for k in ("psi", "ux", "uy", "p", "T", "phi")}
    # the sweep kernel, timed with HIP events on the solver's stream over full launches
    m = case["sweep_block"]
    launch_s = s.time_sweeps(sweep_launches * m) * 1e-3 / sweep_launches
    sweep_kernel = f"k_sweep_tb<{m}, {'double' if precision == 'fp64' else 'float'}, {case['sweep_waves']}, 1>"
    rooflines = {"k_sweep_tb": roofline_of("k_sweep_tb", precision, n, launch_s, workload_name,
                                           SWEEP_COMPULSORY[precision], sweeps=m, shapes=shapes)}
    rooflines["k_sweep_tb"]["kernel"] = sweep_kernel
    rooflines["k_sweep_tb"]["bytes"] = "compulsory: one read and one write of the links and fields per launch"
    # the other kernels of the step (HIP events around back-to-back launches; leaves the state
    # unusable, so this is the last thing done with the solver)
    stage_ms = s.time_stages(5)
    per_step = {"k_sweep_tb": kmean / m * launch_s * 1e3}
    for name, ms in stage_ms.items():
        rooflines[name] = roofline_of(name, precision, n, ms * 1e-3, workload_name, KERNEL_BYTES[name][precision],
                                      shapes=shapes)
        per_step[name] = ms
    stage_total = sum(stage_ms.values()) * 1e-3
    dominant = max(per_step, key=per_step.get)
    del s
    torch.cuda.empty_cache()
    q = np.percentile(sweeps, [0, 10, 50, 90, 100])
    coupled_bytes = (STEP_BYTES[precision] + SWEEP_ELEMS * kmean * ELEM[precision]) * n
    return {
        "value": round(n * steps / dt / 1e6, 3), "ms_per_step": round(ms_step, 4),
        "sweeps_per_step": round(kmean, 2),
        "sweeps_per_step_distribution": {"min": int(q[0]), "p10": float(q[1]), "p50": float(q[2]),
                                         "p90": float(q[3]), "max": int(q[4])},
        "capped_solves_in_timed_steps": int(capped),
        "sweep_mlups": round(n * m / launch_s / 1e6, 1),
        "kernel_ms_per_step": {k: round(v, 4) for k, v in per_step.items()},
        "dominant_kernel": dominant,
        "stage_kernels_hbm_frac_on_method_bytes": round(STEP_BYTES[precision] * n / stage_total / 1e9 / HBM_PEAK_GBS, 4),
        "coupled_hbm_roofline_frac": round(coupled_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "initial_solve": {"sweeps": int(k_init), "seconds": round(init_s, 2), "start": "learned warm start",
                          "converged": True},
        "launch_shapes": shapes,
        "autotune_timings": TUNE_TIMINGS.get((case["nx"], case["ny"], precision)),
        "roofline": rooflines[dominant], "rooflines": rooflines,
        "state": {"step": d["step"], "V_s": d["V_s"], "height": d["height"], "nonfinite": d["nonfinite"],
                  "op_resid_over_ramp": d["op_resid"] / d["op_resid_ramp"] if d["op_resid_ramp"] else None},
        "_fields": fields,
    }


def run_batched(steps, warmup, seed=4, ncases=96, cap=400000):
    """The batched form on the 96-case sweep (uneven grids 256x128 .. 1536x768, FP32), under the
    method's own stopping rule: every case's initial potential is seeded by the learned warm
    start and swept to 1e-8 (lbm_batch_warm_start, lbm_batch_solve_potential), then the whole
    batch advances `steps` timed steps with one launch per stage, against the same cases run
    one at a time with the same start.  `cap` only guards against a runaway solve; the run
    reports how many solves reached it."""
    import numpy as np
    import torch

    from paper_2410_06657_amd import inputs, warm
    from paper_2410_06657_amd.lbm import Batch, Solver, autotune

    cases = inputs.drop_batch(seed, ncases)
    big = max(cases, key=lambda c: c["nx"] * c["ny"])
    tune = autotune(dict(big, poisson_max_sweeps=2000), "fp32", launches=10, persist=False)
    shape = {"sweep_block": tune["sweep_block"], "sweep_waves": tune["sweep_waves"]}
    cases = [dict(c, poisson_max_sweeps=cap, skip_initial_solve=1, **shape) for c in cases]
    # Stage segments: the library's default lowers a small grid's segment height until its own
    # launch has 2048 workgroups; a batch has those many times over, so its cases take 32-row
    # segments (less halo re-reading; 14% faster steps than the per-case default on this
    # batch).  Each case alone keeps the default, which its autotuner finds within a few % of
    # its best.
    batch_cases = [dict(c, stage_rows=BATCH_STAGE_ROWS) for c in cases]
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    factors = [warm.coarse_factor(c["nx"], c["ny"]) for c in cases]
    net = warm.load(max((c["nx"] // f) * (c["ny"] // f) for c, f in zip(cases, factors)))
    t0 = time.perf_counter()
    b = Batch(batch_cases, precision="fp32")
    b.warm_start(net)
    kinit = b.solve_potential()
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    print(f"[bench] batched: {len(cases)} cases, {nodes} nodes, warm-started initial solves "
          f"(up to {kinit} sweeps) {t_init:.1f}s", file=sys.stderr, flush=True)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    logs_b = [b.sweep_log(c) for c in range(len(cases))]
    capped = sum(int(np.sum(lg[1:] >= cap)) for lg in logs_b)
    sw_b = int(sum(int(np.sum(lg[2 + warmup:])) for lg in logs_b))
    del b
    torch.cuda.empty_cache()
    print(f"[bench] batched: {steps} steps in {dt_b:.2f}s", file=sys.stderr, flush=True)
    dt_s, sw_s, t_init_s = 0.0, 0, 0.0
    for k, (c, f) in enumerate(zip(cases, factors)):
        t0 = time.perf_counter()
        s = Solver(c, precision="fp32")
        s.warm_start(net, f)
        s.solve_potential(c["poisson_tol"], cap)
        s.step(warmup)
        torch.cuda.synchronize()
        t_init_s += time.perf_counter() - t0
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        dt_s += time.perf_counter() - t0
        sw_s += int(np.sum(s.sweep_log()[2 + warmup:]))
        del s
        if k % 16 == 15:
            print(f"[bench] one at a time: {k + 1} cases, {dt_s:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return {"value": round(nodes * steps / dt_b / 1e6, 3), "unit": "MLUPS",
            "ms_per_step": round(dt_b / steps * 1e3, 3),
            "one_at_a_time_value": round(nodes * steps / dt_s / 1e6, 3),
            "speedup_vs_one_at_a_time": round(dt_s / dt_b, 3),
            "ncases": len(cases), "nodes": nodes, "steps": steps, "warmup": warmup,
            "stopping_rule": "relative change 1e-8 (every solve)", "capped_solves": capped,
            "initial_solve": {"start": "learned warm start", "max_sweeps": kinit,
                              "batch_seconds": round(t_init, 2)},
            "dtype": "f32", "sweep_shape": shape,
            "stage_rows": {"batched": BATCH_STAGE_ROWS, "one_at_a_time": "library default of each case"},
            "sweeps_total": sw_b, "sweeps_total_one_at_a_time": sw_s,
            "workload": "96 sessile drops, Ny~U{128..768 step 16}, Nx=2Ny, R0=0.3125Ny, "
                        "Ca_E~U[0,0.4], theta~U[45,135], R~logU[0.3,5], S~logU[0.5,3], Ste=0.1, seed 4"}


def finite_or_null(v):
    """The result line as strict JSON: a non-finite float becomes null."""
    if isinstance(v, dict):
        return {k: finite_or_null(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [finite_or_null(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def run_warm(steps=20, seed=6):
    """Learned warm start on the 2048 x 1024 grid (R0 = 320, theta = 90, R = 3, S = 1,
    Ca_E = 0.1): the initial potential solve from the linear ramp
    (cold) against network seed + the same sweeps (warm), both to 1e-8, and the relative L2
    difference of the two potentials (the stopping rule's accuracy: both stop at the same
    relative change, from different sides); then `steps` steps with every solve started from
    the previous step's potential against every solve seeded by the network."""
    import numpy as np
    import torch

    from paper_2410_06657_amd import inputs, warm
    from paper_2410_06657_amd.lbm import Solver

    nx, ny = 2048, 1024
    f = warm.factor_for(ny)
    net = warm.load((nx // f) * (ny // f))
    c = inputs.sessile_drop(nx, ny, 0.3125 * ny, 90.0, 3.0, 1.0, 0.1, 0.1, seed=seed)
    c["poisson_max_sweeps"] = 4000000
    t0 = time.perf_counter()
    cold = Solver(c)
    torch.cuda.synchronize()
    t_cold = time.perf_counter() - t0
    k_cold = int(cold.sweep_log()[0])
    print(f"[bench] warm: cold initial solve {k_cold} sweeps, {t_cold:.2f}s", file=sys.stderr, flush=True)
    w = Solver(dict(c, skip_initial_solve=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w.warm_start(net, f)
    rc, k_warm, _ = w.solve_potential(c["poisson_tol"], c["poisson_max_sweeps"])
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    print(f"[bench] warm: warm initial solve {k_warm} sweeps, {t_warm:.2f}s", file=sys.stderr, flush=True)
    pc, pw = cold.field("phi"), w.field("phi")
    diff = float(np.linalg.norm(pw - pc) / np.linalg.norm(pc))
    # mid-run: the same state stepped with and without the per-step network seed
    res = {}
    for name, s in (("previous_step", cold), ("network", w)):
        if name == "network":
            s.set_warm_start(net, f)
        n0 = len(s.sweep_log())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"ms_per_step": round(dt / steps * 1e3, 3),
                     "sweeps_per_step": round(float(np.mean(s.sweep_log()[n0:])), 2)}
    return {"workload": f"{nx}x{ny} sessile drop, R0=320, theta=90, R=3, S=1, Ca_E=0.1, seed {seed}, FP64",
            "coarse_factor": f,
            "t0": {"cold_sweeps": k_cold, "cold_s": round(t_cold, 3), "warm_sweeps": k_warm,
                   "warm_s": round(t_warm, 3), "speedup": round(t_cold / t_warm, 2),
                   "phi_rel_diff_warm_vs_cold": diff},
            "mid_run": {"steps": steps, **res}}


def run_validation():
    """The paper's validation problems (Sec. 4) and its electrofreezing study (Sec. 5) as FP64
    batches: the Fig. 5 deformation sweeps (12 free drops, R0 = 20 in 160 x 160, 10,000 steps),
    the Neumann front at four Stefan numbers, the final height of six freezing layers (with the
    largest deviations from the closed forms), and 24 wetting drops frozen with and without
    the field; wall time of each."""
    import torch

    from paper_2410_06657_amd import validation as v

    out = {}
    t0 = time.perf_counter()
    d = v.deformation_sweep()
    torch.cuda.synchronize()
    out["deformation"] = {
        "workload": "12 free drops, R0=20 in 160x160, Ca_E=0.2, R=5 with S in 1..15 and S=2 with R in 0.5..8, FP64 batch, D averaged over steps 6000-10000",
        "wall_s": round(time.perf_counter() - t0, 2),
        "points": [{k: (round(x, 5) if isinstance(x, float) else x) for k, x in r.items()} for r in d],
        "sign_agrees_with_feng": all((r["D"] > 0) == (r["feng"] > 0) for r in d),
        "max_outside_taylor_feng_band": round(max(max(min(r["feng"], r["taylor"]) - r["D"],
                                                      r["D"] - max(r["feng"], r["taylor"]), 0.0) for r in d), 5)}
    print(f"[bench] validation: deformation sweep {out['deformation']['wall_s']}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    nm = v.neumann_sweep()
    out["neumann_front"] = {"workload": "4x48 strips, alpha_s=0.2, Ste in {0.05, 0.1, 0.2, 0.5}, FP64 batch",
                            "wall_s": round(time.perf_counter() - t0, 2),
                            "max_rel_err": round(max(max(r["rel_err"]) for r in nm), 5)}
    t0 = time.perf_counter()
    fh = v.final_height_sweep()
    out["final_height"] = {"workload": "4x48 strips, h0=16, Ste in {0.2, 0.5} x rho_s/rho_l in {0.9, 1.0, 1.1}, FP64 batch",
                           "wall_s": round(time.perf_counter() - t0, 2),
                           "max_rel_err": round(max(abs(r["h_f_over_h_0"] / r["closed_form"] - 1) for r in fh), 5)}
    print(f"[bench] validation: Stefan sweeps {out['neumann_front']['wall_s']}s + {out['final_height']['wall_s']}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ps = v.parameter_study()
    out["parameter_study"] = {
        "workload": "24 sessile drops, R0=20 in 160x80, theta=120, modes none/PR+(2,0.5)/OB-(2,5)/PR-(5,9.5) at Ca_E=1, "
                    "Ste in {0.05, 0.1, 0.2}, rho_s/rho_l in {0.9, 1.1}, each to its freezing time, FP64 batch",
        "wall_s": round(time.perf_counter() - t0, 2),
        "rows": [{"rho_s_over_rho_l": r["rho_s_over_rho_l"], "Ste": r["Ste"], "mode": r["mode"],
                  "t_fre": round(r["t_fre"], 1), "H_m_over_H_0": round(r["H_m_over_H_0"], 4),
                  "t_star": round(r["t_star"], 4),
                  "substrate_flux": {"first": {"Fo": round(r["substrate_flux"][0][0], 3),
                                               "flux": float(f"{r['substrate_flux'][0][1]:.4g}")},
                                     "last": {"Fo": round(r["substrate_flux"][-1][0], 3),
                                              "flux": float(f"{r['substrate_flux'][-1][1]:.4g}")}}}
                 for r in ps],
        "ste_fo_law": {k: round(v, 4) for k, v in v.ste_fo_law(ps).items()}}
    print(f"[bench] validation: parameter study {out['parameter_study']['wall_s']}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    cw = v.cold_wall()
    out["cold_wall"] = {
        "workload": "water and hexadecane drops (Table 1 ratios), R0=20 in 160x80, theta=87, frozen completely, FP64 batch",
        "wall_s": round(time.perf_counter() - t0, 2),
        "rows": [{k: (round(float(x), 5) if isinstance(x, float) else x) for k, x in r.items()} for r in cw]}
    print(f"[bench] validation: cold wall {out['cold_wall']['wall_s']}s", file=sys.stderr, flush=True)
    return out


TTF_GRIDS = {"128x64": (128, 64, 24.0), "512x256": (512, 256, 96.0), "1024x512": (1024, 512, 192.0)}
# grids whose time to freeze is measured for the single-case precision forms only (at 50-70 s
# per drop, the warm start, the two batches of 8 and the 8 seeds one at a time would add some
# 15-20 minutes)
TTF_FORMS_ONLY = {"1024x512"}


def run_time_to_freeze(nbatch=8, max_steps=1000000, grid="128x64", tune=True):
    """Time to freeze (R30) of a sessile drop (128 x 64 with R0 = 24, or the same drop four times
    larger, 512 x 256 with R0 = 96; theta = 90, R = 3, S = 1, Ca_E = 0.1, Ste = 0.1): FP64,
    FP32, FP32 with FP16 population storage, FP64 with the learned warm start of the initial
    potential, `nbatch` seeds (centre jitter) in one FP32 batch against the same seeds one
    at a time, and the same seeds as one FP16-storage batch.  Speedups are quoted with the
    freezing times they reach.  Every run takes its precision's autotuned sweep shape (the
    batches too; tune=False: the library defaults), which changes no result.  On the
    1024 x 512 drop (R0 = 192) only FP64, FP32 and FP16 storage run."""
    import torch

    from paper_2410_06657_amd import inputs, warm
    from paper_2410_06657_amd.lbm import Batch, Solver

    def one(case, precision, net=None, factor=0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if net is None:
            s = Solver(case, precision)
        else:
            s = Solver(dict(case, skip_initial_solve=1), precision)
            s.warm_start(net, factor)
            s.solve_potential(case["poisson_tol"], case["poisson_max_sweeps"])
        k = s.run_until_frozen(max_steps, 20)  # t_fre is detected on the device; the host looks every 20 steps
        torch.cuda.synchronize()
        return time.perf_counter() - t0, s.diag()["t_fre"], k

    nx, ny, r0 = TTF_GRIDS[grid]
    base = lambda sd: inputs.sessile_drop(nx, ny, r0, 90.0, 3.0, 1.0, 0.1, 0.1, seed=sd)
    # the sweep shape of each precision (timed before any clock starts)
    sweep = {}
    for p in ("fp64", "fp32", "fp16store"):
        sh = launch_shapes(base(0), p, tune)
        sweep[p] = {"sweep_block": sh["sweep_block"], "sweep_waves": sh["sweep_waves"]}
    mk = lambda sd, p="fp32": dict(base(sd), **sweep[p])
    out = {"workload": f"{grid} sessile drop, R0={r0:g}, theta=90, R=3, S=1, Ca_E=0.1, Ste=0.1, seed 0",
           "sweep_shapes": sweep,
           "autotune_us_per_sweep": {p: (TUNE_TIMINGS.get((nx, ny, p)) or {}).get("us_per_sweep") for p in sweep}}
    t64, f64, k64 = one(mk(0, "fp64"), "fp64")
    print(f"[bench] time to freeze {grid}: fp64 {t64:.2f}s ({k64} steps)", file=sys.stderr, flush=True)
    t32, f32, _ = one(mk(0, "fp32"), "fp32")
    print(f"[bench] time to freeze {grid}: fp32 {t32:.2f}s", file=sys.stderr, flush=True)
    t16, f16, _ = one(mk(0, "fp16store"), "fp16store")
    print(f"[bench] time to freeze {grid}: fp16 storage {t16:.2f}s", file=sys.stderr, flush=True)
    out["fp64"] = {"wall_s": round(t64, 3), "t_fre": f64, "steps": k64}
    out["fp32"] = {"wall_s": round(t32, 3), "t_fre": f32, "t_fre_rel_diff": abs(f32 - f64) / f64,
                   "speedup_vs_fp64": round(t64 / t32, 3)}
    out["fp16store"] = {"wall_s": round(t16, 3), "t_fre": f16, "t_fre_rel_diff": abs(f16 - f64) / f64,
                        "speedup_vs_fp64": round(t64 / t16, 3)}
    if grid in TTF_FORMS_ONLY:
        return out
    f = warm.factor_for(ny)
    net = warm.load((nx // f) * (ny // f))
    tw, fw, _ = one(mk(0, "fp64"), "fp64", net, f)
    out["warm_fp64"] = {"wall_s": round(tw, 3), "t_fre": fw, "t_fre_rel_diff": abs(fw - f64) / f64,
                        "speedup_vs_fp64": round(t64 / tw, 3)}
    print(f"[bench] time to freeze: fp64 {t64:.2f}s, fp32 {t32:.2f}s, fp16 storage {t16:.2f}s, warm {tw:.2f}s",
          file=sys.stderr, flush=True)
    cases = [mk(sd) for sd in range(nbatch)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = Batch(cases, precision="fp32")
    b.run_until_frozen(max_steps)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    fb = [d["t_fre"] for d in b.diag()]
    del b
    ts, fs = 0.0, []
    for k, case in enumerate(cases):
        dt, fr, _ = one(case, "fp32")
        ts += dt
        fs.append(fr)
        print(f"[bench] time to freeze: seed {k} alone {dt:.2f}s", file=sys.stderr, flush=True)
    out["batched_fp32"] = {"cases": nbatch, "wall_s": round(tb, 3), "one_at_a_time_wall_s": round(ts, 3),
                           "speedup_vs_one_at_a_time": round(ts / tb, 3),
                           "t_fre_rel_diff_vs_fp64_seed0": abs(fb[0] - f64) / f64,
                           "t_fre_equal_to_single_runs": fb == fs}
    print(f"[bench] time to freeze: batch of {nbatch} {tb:.2f}s, one at a time {ts:.2f}s", file=sys.stderr, flush=True)
    # the same seeds as one batch with FP16 population storage (seed 0's single run: above)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = Batch([mk(sd, "fp16store") for sd in range(nbatch)], precision="fp16store")
    b.run_until_frozen(max_steps)
    torch.cuda.synchronize()
    th = time.perf_counter() - t0
    fh = [d["t_fre"] for d in b.diag()]
    del b
    out["batched_fp16store"] = {"cases": nbatch, "wall_s": round(th, 3),
                                "speedup_vs_fp32_batch": round(tb / th, 3),
                                "t_fre_rel_diff_vs_fp64_seed0": abs(fh[0] - f64) / f64,
                                "seed0_t_fre_equal_to_single_run": fh[0] == f16}
    print(f"[bench] time to freeze: FP16-storage batch of {nbatch} {th:.2f}s", file=sys.stderr, flush=True)
    return out


def counters_probe(case, launches=20, tune=True):
    """Short run for hardware-counter passes (rocprofv3 --pmc): a plain copy kernel of known
    size (the calibration of the byte counters), then `launches` blocked sweep launches and
    three steps per precision (FP64, FP32, FP16 storage) on the workload's grid, with the
    launch shapes the benchmark takes (printed).  The initial potential solve is capped at 16
    sweeps so the run stays short; a launch's memory traffic does not depend on convergence."""
    import torch

    from paper_2410_06657_amd.lbm import Solver

    nbytes = 256 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[counters] copy kernel: 3 x {nbytes} bytes read and written", file=sys.stderr, flush=True)
    del src, dst
    for precision in ("fp64", "fp32", "fp16store"):
        shapes = launch_shapes(case, precision, tune)
        print(f"[counters] launch_shapes {precision} {shapes['sweep_block']} {shapes['sweep_waves']} "
              f"{shapes['stage_rows']}", file=sys.stderr, flush=True)
        c = dict(case, poisson_max_sweeps=16, poisson_tol=-1.0, **shapes)
        m = c["sweep_block"]
        s = Solver(c, precision=precision)
        s.time_sweeps(launches * m)
        s.step(3)  # the stage kernels of a step (with 16-sweep solves)
        torch.cuda.synchronize()
        print(f"[counters] {precision}: {launches} launches of {m} sweeps and 3 steps on {c['nx']}x{c['ny']}",
              file=sys.stderr, flush=True)
        del s


def nn_probe(iters=10, batch=64, h=32, w=64):
    """Short run of the warm-start network's kernels for a kernel trace: `iters` training steps
    (forward, backward, Adam) and `iters` forward passes on `batch` random 32 x 64 maps."""
    import torch

    from paper_2410_06657_amd.lbm import Net
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn((batch, h, w, 3), generator=g, device="cuda")
    t = torch.randn((batch, h, w), generator=g, device="cuda") * 0.1
    net = Net(batch * h * w, seed=2)
    for _ in range(iters):
        net.train_step(x, t, 1e-3)
    for _ in range(iters):
        net.forward(x)
    torch.cuda.synchronize()
    print(f"[nn-probe] {iters} training steps and {iters} forward passes on {batch} x {h} x {w} pixels",
          file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="4096x2048")
    ap.add_argument("--sweep-launches", type=int, default=50,
                    help="blocked sweep launches timed with HIP events for the sweep kernel's roofline")
    ap.add_argument("--init-cap", type=int, default=4000000,
                    help="sweep cap of the warm-started initial potential solve (the run fails if it is reached)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 forms (FP32 and FP16 storage)")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default launch shapes instead of the autotuner's (sweeps 8 x 4 waves, "
                         "default stage rows)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched form")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm start comparison")
    ap.add_argument("--no-time-to-freeze", action="store_true", help="skip the time-to-freeze runs")
    ap.add_argument("--time-to-freeze-grid", default="128x64", choices=sorted(TTF_GRIDS),
                    help="drop of the time-to-freeze runs (512x256: the same drop four times larger)")
    ap.add_argument("--time-to-freeze-only", action="store_true",
                    help="print only the time-to-freeze runs as one JSON object")
    ap.add_argument("--batched-only", action="store_true", help="print only the batched form as one JSON object")
    ap.add_argument("--no-validation", action="store_true", help="skip the validation problems")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--counters", action="store_true",
                    help="short run for rocprofv3 --pmc passes (copy calibration + sweep launches)")
    ap.add_argument("--nn-probe", action="store_true",
                    help="short run of the warm-start network's kernels (for a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.nn_probe:
        nn_probe()
        return
    if args.batched_only:
        print(json.dumps(finite_or_null(run_batched(args.batched_steps, 2)), allow_nan=False), flush=True)
        return
    if args.time_to_freeze_only:
        print(json.dumps(finite_or_null(run_time_to_freeze(grid=args.time_to_freeze_grid, tune=not args.no_tune)),
                         allow_nan=False),
              flush=True)
        return
    case, desc = workload(args.workload)
    if args.counters:
        counters_probe(case, tune=not args.no_tune)
        return
    import numpy as np

    from paper_2410_06657_amd import warm
    n = case["nx"] * case["ny"]
    factor = warm.factor_for(case["ny"])
    net = warm.load((case["nx"] // factor) * (case["ny"] // factor))
    run = lambda prec: run_form(case, prec, args.steps, args.warmup, args.sweep_launches, args.workload,
                                net, factor, args.init_cap, tune=not args.no_tune)
    f64 = run("fp64")
    ref = f64.pop("_fields")
    line = {
        "metric": METRIC, "value": f64["value"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "nx": case["nx"], "ny": case["ny"], "precision": "fp64",
                   "poisson_tol": case["poisson_tol"], "launch_shapes": f64.get("launch_shapes"),
                   "initial_potential": "learned warm start, then sweeps to the same stopping rule"},
        "sweeps_per_step": f64["sweeps_per_step"],
        "sweeps_per_step_distribution": f64["sweeps_per_step_distribution"],
        "capped_solves_in_timed_steps": f64["capped_solves_in_timed_steps"],
        "sweep_mlups": f64["sweep_mlups"],
        "kernel_ms_per_step": f64["kernel_ms_per_step"],
        "dominant_kernel": f64["dominant_kernel"],
        "stage_kernels_hbm_frac_on_method_bytes": f64["stage_kernels_hbm_frac_on_method_bytes"],
        "coupled_hbm_roofline_frac": f64["coupled_hbm_roofline_frac"],
        "initial_solve": f64["initial_solve"],
        "roofline": f64["roofline"],
        "rooflines": f64["rooflines"],
        "hbm_copy": copy_bandwidth(),
        "state": f64["state"],
    }
    if not args.no_fp32:
        line["forms"] = {}
        for prec in ("fp32", "fp16store"):
            r = run(prec)
            cur = r.pop("_fields")
            r["speedup_vs_fp64"] = round(r["value"] / f64["value"], 3)
            r["rel_l2_vs_fp64_after_timed_steps"] = {
                k: float(np.linalg.norm(cur[k] - ref[k]) / max(np.linalg.norm(ref[k]), 1e-300)) for k in ref}
            line["forms"][prec] = r
    if not args.no_time_to_freeze:
        line["time_to_freeze"] = run_time_to_freeze(grid=args.time_to_freeze_grid, tune=not args.no_tune)
    if not args.no_validation:
        line["validation"] = run_validation()
    if not args.no_warm:
        line.setdefault("forms", {})["warm"] = run_warm()
    if not args.no_batched:
        line.setdefault("forms", {})["batched"] = run_batched(args.batched_steps, 2)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(case, f64["sweeps_per_step"])
        cb.pop("step_s")
        line["cpu_baseline"] = cb
    print(json.dumps(finite_or_null(line), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
