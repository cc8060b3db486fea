"""Batched form: every case of a batch advanced with one launch per stage (stages outside
the potential loop replayed from HIP graphs) equals its own single-case run bitwise, in
FP64, in FP32 and with FP16 population storage, and the FP64 batch equals the oracle to the
FP64 bar."""
import math
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu


def mixed_cases():
    """Five cases of different sizes, angles and electric ratios (ragged tiles included)."""
    return [
        inputs.sessile_drop(96, 48, 16, 60.0, 3.0, 1.0, 0.2, 0.2, seed=1),
        inputs.sessile_drop(128, 64, 24, 90.0, 0.5, 2.0, 0.3, 0.1, seed=2),
        inputs.sessile_drop(200, 100, 30, 120.0, 2.0, 5.0, 0.4, 0.2, seed=3, rho_ratio_sl=1.1),
        inputs.stefan_strip(4, 40, h0=20.0, Ste=0.3, rho_ratio_sl=0.9),
        inputs.sessile_drop(70, 45, 14, 75.0, 5.0, 2.0, 0.1, 0.2, seed=5),
    ]


@pytest.mark.parametrize("precision,shape", [("fp64", (8, 4)), ("fp32", (8, 4)), ("fp32", (4, 8)),
                                             ("fp16store", (8, 4)), ("fp64", (16, 8)), ("fp32", (16, 8))])
def test_batch_equals_single_runs(precision, shape):
    from paper_2410_06657_amd.lbm import Batch, Solver
    cases = [dict(c, sweep_block=shape[0], sweep_waves=shape[1]) for c in mixed_cases()]
    b = Batch(cases, precision=precision)
    b.step(15)
    for c, case in enumerate(cases):
        s = Solver(case, precision=precision)
        s.step(15)
        assert list(b.sweep_log(c)) == list(s.sweep_log()), c
        for k in ("psi", "ux", "uy", "p", "T", "H", "fs", "phi"):
            assert np.array_equal(b.field(c, k), s.field(k)), (c, k)
        print(f"case {c} {case['nx']}x{case['ny']} equal", flush=True)


def test_batch_fp64_matches_oracle():
    from paper_2410_06657_amd.lbm import Batch
    ob.set_threads(min(16, os.cpu_count() or 1))
    cases = mixed_cases()[:3]
    b = Batch(cases, precision="fp64")
    b.step(10)
    for c, case in enumerate(cases):
        o = ob.Oracle(case)
        o.step(10)
        assert list(b.sweep_log(c)) == list(o.sweep_log()), c
        for k in ("psi", "ux", "p", "T", "phi"):
            a, r = b.field(c, k), o.field(k)
            err = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-12 * math.sqrt(r.size))
            assert err <= 1e-10, (c, k, err)


def test_batch_freezing_times():
    """Strips of different heights and undercoolings freeze completely inside one batch; the
    on-device freezing-time detector of every case equals its single-case value."""
    from paper_2410_06657_amd.lbm import Batch, Solver
    cases = [inputs.stefan_strip(4, 24 + 8 * k, h0=8.0 + 2 * k, Ste=0.4 + 0.1 * k, rho_ratio_sl=0.9)
             for k in range(4)]
    b = Batch(cases, precision="fp64")
    b.step(1500)
    d = b.diag()
    for c, case in enumerate(cases):
        s = Solver(case)
        s.step(1500)
        ds = s.diag()
        assert ds["t_fre"] > 0, c
        assert d[c]["t_fre"] == ds["t_fre"], c
        assert d[c]["V_s"] == ds["V_s"], c


@pytest.mark.parametrize("precision", ["fp64", "fp16store"])
def test_batch_run_until_frozen_matches_single_runs(precision):
    """Cases freezing at different steps: each stops at its own freezing step inside the batch
    (its workgroups idle from then on) and ends bitwise where its single-case run stops (with
    FP16 storage too: every case keeps its own binary16 scales)."""
    from paper_2410_06657_amd.lbm import Batch, Solver
    cases = [inputs.stefan_strip(4, 24 + 8 * k, h0=8.0 + 2 * k, Ste=0.4 + 0.1 * k, rho_ratio_sl=0.9)
             for k in range(3)]
    cases.append(inputs.sessile_drop(64, 32, 10.0, 90.0, 3.0, 1.0, 0.1, 0.5, seed=5))
    b = Batch(cases, precision=precision)
    nb = b.run_until_frozen(5000)
    d = b.diag()
    steps = []
    for c, case in enumerate(cases):
        s = Solver(case, precision=precision)
        k = s.run_until_frozen(5000, 1)
        ds = s.diag()
        steps.append(k)
        assert ds["t_fre"] > 0 and d[c]["t_fre"] == ds["t_fre"], c
        assert d[c]["step"] == ds["step"] == k, c
        assert list(b.sweep_log(c)) == list(s.sweep_log()), c
        for name in ("psi", "T", "fs", "phi", "ux"):
            assert np.array_equal(b.field(c, name), s.field(name)), (c, name)
    print("freezing steps", steps, "batch steps", nb)
    assert nb == max(steps) and len(set(steps)) > 1


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16store"])
def test_batch_warm_start_equals_single_runs(precision):
    """Cases initialised without a solve, seeded by the learned warm start in one batch call
    (each with its own coarse factor) and solved to the stopping rule in lockstep, then stepped:
    every case equals its single-case run with the same start, bitwise."""
    from paper_2410_06657_amd import warm
    from paper_2410_06657_amd.lbm import Batch, Solver
    cases = [dict(c, skip_initial_solve=1) for c in mixed_cases() if c["nx"] > 4]
    factors = [warm.coarse_factor(c["nx"], c["ny"]) for c in cases]
    net = warm.load(max((c["nx"] // f) * (c["ny"] // f) for c, f in zip(cases, factors)))
    b = Batch(cases, precision=precision)
    b.warm_start(net)
    kmax = b.solve_potential()
    b.step(5)
    for c, (case, f) in enumerate(zip(cases, factors)):
        s = Solver(case, precision=precision)
        s.warm_start(net, f)
        s.solve_potential(case["poisson_tol"], case["poisson_max_sweeps"])
        s.step(5)
        assert list(b.sweep_log(c)) == list(s.sweep_log()), c
        assert b.sweep_log(c)[1] <= kmax
        for k in ("psi", "ux", "uy", "p", "T", "H", "fs", "phi"):
            assert np.array_equal(b.field(c, k), s.field(k)), (c, k)
        print(f"case {c} {case['nx']}x{case['ny']} factor {f}: equal, initial solve {int(s.sweep_log()[1])} sweeps",
              flush=True)
