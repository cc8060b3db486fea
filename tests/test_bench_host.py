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


def test_traffic_only_for_the_profiled_source(monkeypatch):
    t64, t32 = bench.measured_traffic("fp64", "1024x512"), bench.measured_traffic("fp32", "1024x512")
    if t64 is None:
        pytest.skip("the committed counter summary was taken from another kernel source")
    # above the compulsory bytes of a launch at 1024 x 512, below twice them
    n = 1024 * 512
    assert bench.SWEEP_COMPULSORY["fp64"] * n <= t64 < 2 * bench.SWEEP_COMPULSORY["fp64"] * n
    assert bench.SWEEP_COMPULSORY["fp32"] * n <= t32 < 2 * bench.SWEEP_COMPULSORY["fp32"] * n
    assert bench.measured_traffic("fp16store", "1024x512") == t32
    assert bench.measured_traffic("fp64", "128x64") is None
    monkeypatch.setattr(bench, "sweep_source_digest", lambda: "0" * 64)
    assert bench.measured_traffic("fp64", "1024x512") is None


def test_main_line_contract(monkeypatch, capsys):
    """The JSON line's keys, with the GPU measurement replaced by a stand-in of the same shape."""
    import json

    def fake_form(case, precision, steps, warmup, sweep_launches, workload_name="1024x512"):
        return {"value": 1000.0, "ms_per_step": 0.5, "sweeps_per_step": 80.0,
                "sweeps_per_step_distribution": {"min": 70, "p10": 72.0, "p50": 80.0, "p90": 90.0, "max": 95},
                "sweep_mlups": 2e5, "sweep_time_share": 0.5, "coupled_hbm_roofline_frac": 1.0,
                "coupled_algorithmic_GBs": 8000.0, "init_s": 1.0,
                "roofline": {"bound": "hbm", "achieved": 1.0, "peak": 8000.0, "unit": "GB/s", "frac": 1.25e-4,
                             "traffic": None},
                "state": {"step": 65, "V_s": 0.0, "height": 1.0, "nonfinite": 0}}

    monkeypatch.setattr(bench, "run_form", fake_form)
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-fp32", "--no-time-to-freeze", "--no-validation",
                                      "--no-warm", "--no-batched", "--no-cpu-baseline"])
    bench.main()
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "sweeps_per_step",
              "sweeps_per_step_distribution", "sweep_mlups"):
        assert k in line, k
    assert line["n_gpus"] == 1 and line["config"]["nx"] == 1024 and line["dtype"] == "f64"
    assert set(line["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}


def test_host_cpu():
    h = bench.host_cpu()
    assert h["nproc"] >= 1
    assert h["cpu_model"] is None or isinstance(h["cpu_model"], str)
