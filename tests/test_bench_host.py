"""Host logic of bench.py (no GPU): the one-GPU guard, the byte models of the roofline
figures and the rule that measured traffic is reported only for the kernel source it was
taken from."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_models():
    # a potential sweep moves 4 links, phi and 1/tau_l in and 4 links and phi out
    assert bench.SWEEP_ELEMS * bench.ELEM["fp64"] == 88
    assert bench.SWEEP_ELEMS * bench.ELEM["fp32"] == 44
    # outside the sweeps: 27 + 27 populations and 13 + 13 fields per node and step
    assert bench.STEP_BYTES["fp64"] == 640 and bench.STEP_BYTES["fp32"] == 320
    # FP16 storage: the populations in 2 bytes, the fields in 4
    assert bench.STEP_BYTES["fp16store"] == 54 * 2 + 26 * 4 == 212
    # the FP16-storage form sweeps FP32 links
    assert bench.ELEM["fp16store"] == 4 and bench.SWEEP_COMPULSORY["fp16store"] == bench.SWEEP_COMPULSORY["fp32"]


def test_traffic_only_for_the_profiled_source(monkeypatch, tmp_path):
    """Counter bytes are reported only from a summary of the same workload and kernel source."""
    f = tmp_path / "c.md"
    f.write_text(f"kernel_source_sha256 {bench.kernel_source_digest()}\n"
                 "traffic_bytes_per_launch k_h_stream fp64 123456\n")
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    assert bench.measured_traffic("k_h_stream", "fp64", "4096x2048") == 123456
    assert bench.measured_traffic("k_h_stream", "fp32", "4096x2048") is None
    assert bench.measured_traffic("k_h_stream", "fp64", "1024x512") is None
    # with the launch shapes it was taken with on record, other shapes get no figure
    f.write_text(f"kernel_source_sha256 {bench.kernel_source_digest()}\n"
                 "launch_shapes fp64 8 4 32\n"
                 "traffic_bytes_per_launch k_h_stream fp64 123456\n")
    same = {"sweep_block": 8, "sweep_waves": 4, "stage_rows": 32}
    assert bench.measured_traffic("k_h_stream", "fp64", "4096x2048", same) == 123456
    assert bench.measured_traffic("k_h_stream", "fp64", "4096x2048", dict(same, stage_rows=16)) is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    assert bench.measured_traffic("k_h_stream", "fp64", "4096x2048") is None


def test_kernel_byte_tables():
    # the kernels of a step together move more than the method's minimum (intermediate planes)
    for prec in ("fp64", "fp32", "fp16store"):
        assert sum(v[prec] for v in bench.KERNEL_BYTES.values()) >= bench.STEP_BYTES[prec]
    # g: 18 populations; H, T, psi (2 levels), f_s, u (2 levels x 2), mdot in; H, T, f_s, mdot,
    # f_l, psi u (2) out
    assert bench.KERNEL_BYTES["k_g_stream"]["fp64"] == 18 * 8 + 17 * 8
    # h: 18 populations; psi, f_s, phi, p, u (2), u* (2), mdot in; p, u (2), u* (2) out
    assert bench.KERNEL_BYTES["k_h_fused"]["fp64"] == 18 * 8 + 14 * 8


def test_main_line_contract(monkeypatch, capsys):
    """The JSON line's keys, with the GPU measurement replaced by a stand-in of the same shape."""
    import json
    import types

    import numpy as np

    def fake_form(case, precision, steps, warmup, sweep_launches, workload_name, net, factor, init_cap, tune=True):
        rl = {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 1.25e-4, "traffic": None}
        return {"value": 1000.0, "ms_per_step": 0.5, "sweeps_per_step": 10.0,
                "sweeps_per_step_distribution": {"min": 9, "p10": 9.0, "p50": 10.0, "p90": 11.0, "max": 12},
                "capped_solves_in_timed_steps": 0, "sweep_mlups": 2e5,
                "kernel_ms_per_step": {"k_h_stream": 0.5}, "dominant_kernel": "k_h_stream",
                "stage_kernels_hbm_frac_on_method_bytes": 0.5, "coupled_hbm_roofline_frac": 0.5,
                "initial_solve": {"sweeps": 1000, "seconds": 1.0, "start": "learned warm start", "converged": True},
                "roofline": rl, "rooflines": {"k_h_stream": rl},
                "state": {"step": 45, "V_s": 0.0, "height": 1.0, "nonfinite": 0, "op_resid_over_ramp": 0.05},
                "_fields": {"psi": np.zeros((2, 2))}}

    monkeypatch.setattr(bench, "run_form", fake_form)
    monkeypatch.setattr(bench, "copy_bandwidth", lambda: {"achieved": 1.0, "unit": "GB/s"})
    monkeypatch.setitem(sys.modules, "paper_2410_06657_amd.warm",
                        types.SimpleNamespace(factor_for=lambda ny: 64, load=lambda px: None))
    import paper_2410_06657_amd
    monkeypatch.setattr(paper_2410_06657_amd, "warm", sys.modules["paper_2410_06657_amd.warm"], raising=False)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-fp32", "--no-time-to-freeze", "--no-validation",
                                      "--no-warm", "--no-batched", "--no-cpu-baseline"])
    bench.main()
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "sweeps_per_step",
              "sweeps_per_step_distribution", "sweep_mlups", "rooflines", "initial_solve"):
        assert k in line, k
    assert line["n_gpus"] == 1 and line["config"]["nx"] == 4096 and line["dtype"] == "f64"
    assert set(line["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}


def test_host_cpu():
    h = bench.host_cpu()
    assert h["nproc"] >= 1
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)


def test_untuned_launch_shapes_are_the_library_defaults():
    """bench.py --no-tune takes the shapes a handle takes by default (host-only query), the
    same the committed counter summary records for 4096 x 2048."""
    from paper_2410_06657_amd import inputs
    shapes = bench.launch_shapes(inputs.drop_4096x2048(), "fp64", tune=False)
    assert shapes == {"sweep_block": 8, "sweep_waves": 4, "stage_rows": 32}
    assert bench.shape_key(shapes) == (8, 4, 32)


@pytest.mark.parametrize("grid", ["128x64", "1024x512"])
def test_time_to_freeze_legs(monkeypatch, grid):
    """run_time_to_freeze with stand-in solvers: every form runs the drop of the chosen grid with
    its precision's sweep shape; the 1024 x 512 drop runs the three precision forms only, the
    smaller ones also the warm start and the two batches; speedups are wall-time ratios."""
    import types

    import paper_2410_06657_amd
    from paper_2410_06657_amd import lbm

    made = []

    class FakeSolver:
        def __init__(self, case, precision="fp64"):
            made.append((case["nx"], case["ny"], precision, case["sweep_block"], case["sweep_waves"]))
            self.t = {"fp64": 100.0, "fp32": 100.01, "fp16store": 100.02}[precision]

        def warm_start(self, net, factor):
            pass

        def solve_potential(self, tol, cap):
            pass

        def run_until_frozen(self, max_steps, every):
            return 1234

        def diag(self):
            return {"t_fre": self.t}

    class FakeBatch:
        def __init__(self, cases, precision="fp32"):
            self.n, self.t = len(cases), {"fp32": 100.01, "fp16store": 100.02}[precision]

        def run_until_frozen(self, max_steps):
            pass

        def diag(self):
            return [{"t_fre": self.t}] * self.n

    shapes = {"fp64": (8, 4), "fp32": (16, 8), "fp16store": (8, 8)}
    monkeypatch.setattr(bench, "launch_shapes", lambda case, p, tune=True: {
        "sweep_block": shapes[p][0], "sweep_waves": shapes[p][1], "stage_rows": 32})
    monkeypatch.setattr(lbm, "Solver", FakeSolver)
    monkeypatch.setattr(lbm, "Batch", FakeBatch)
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    fake_warm = types.SimpleNamespace(factor_for=lambda ny: 4, load=lambda px: None)
    monkeypatch.setitem(sys.modules, "paper_2410_06657_amd.warm", fake_warm)
    monkeypatch.setattr(paper_2410_06657_amd, "warm", fake_warm, raising=False)
    out = bench.run_time_to_freeze(nbatch=3, grid=grid)
    nx, ny, _ = bench.TTF_GRIDS[grid]
    assert all((c[0], c[1]) == (nx, ny) for c in made)
    assert all((c[3], c[4]) == shapes[c[2]] for c in made)
    assert out["sweep_shapes"]["fp32"] == {"sweep_block": 16, "sweep_waves": 8}
    assert out["fp64"]["steps"] == 1234
    assert out["fp32"]["t_fre_rel_diff"] == pytest.approx(1e-4)
    assert out["fp32"]["speedup_vs_fp64"] > 0
    if grid == "1024x512":
        assert set(out) == {"workload", "sweep_shapes", "autotune_us_per_sweep", "fp64", "fp32", "fp16store"}
        assert len(made) == 3
    else:
        assert {"warm_fp64", "batched_fp32", "batched_fp16store"} <= set(out)
        assert out["batched_fp32"]["t_fre_equal_to_single_runs"] is True
        assert out["batched_fp16store"]["seed0_t_fre_equal_to_single_run"] is True
        assert len(made) == 4 + 3  # three forms, the warm start, the seeds one at a time
