"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle on the same
seeded inputs.  FP64 bar: relative L2 error <= 1e-10 per field; potential sweep counts
equal step by step."""
import math
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10
FIELDS = ["psi", "ux", "uy", "usx", "usy", "p", "T", "H", "fs", "mdot", "psiu_x", "psiu_y", "phi", "fl"]


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    ob.set_threads(min(16, os.cpu_count() or 1))
    yield
    ob.set_threads(1)


def rel_l2(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    den = max(np.linalg.norm(b), 1e-12 * math.sqrt(b.size))
    return np.linalg.norm(a - b) / den


def solver(case):
    from paper_2410_06657_amd.lbm import Solver
    return Solver(case)


def compare(g, o, fields=FIELDS, tol=TOL, pops=True):
    errs = {}
    for k in fields:
        errs[k] = rel_l2(g.field(k), o.field(k))
    if pops:
        for k in ("f", "h", "g"):
            errs["pop_" + k] = rel_l2(g.pop(k), o.pop(k))
        errs["pop_l"] = rel_l2(g.pop("l"), o.pop("l")[1:])
    print({k: f"{v:.2e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"fields above {tol}: {bad}"
    return errs


def small_drop(seed=0, nx=128, ny=64):
    c = inputs.drop_128x64(seed)
    if (nx, ny) != (128, 64):
        c = inputs.scaled(c, nx, ny)
    return c


def test_init_matches_oracle():
    c = small_drop(0)
    g, o = solver(c), ob.Oracle(c)
    assert list(g.sweep_log()) == list(o.sweep_log())
    compare(g, o)


def test_fixed_sweep_count_matches():
    c = small_drop(1)
    c.update(poisson_max_sweeps=37, poisson_tol=-1.0)
    g, o = solver(c), ob.Oracle(c)
    for _ in range(3):
        rc_g, k_g, r_g = g.solve_potential(-1.0, 13)
        rc_o, k_o, r_o = o.solve_potential(-1.0, 13)
        assert (rc_g, k_g) == (rc_o, k_o) == (0, 13)
        assert r_g == pytest.approx(r_o, rel=1e-9)
    compare(g, o, fields=["phi"], tol=1e-12, pops=False)
    assert rel_l2(g.pop("l"), o.pop("l")[1:]) <= 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ten_steps_128x64(seed):
    c = small_drop(seed)
    g, o = solver(c), ob.Oracle(c)
    g.step(10)
    o.step(10)
    assert list(g.sweep_log()) == list(o.sweep_log())
    compare(g, o)


def test_thousand_steps_128x64():
    """The 128 x 64 sessile-drop workload, 1000 steps, potential to 1e-8 every step."""
    c = small_drop(0)
    g, o = solver(c), ob.Oracle(c)
    for chunk in range(10):
        g.step(100)
        o.step(100)
        assert list(g.sweep_log()) == list(o.sweep_log()), f"sweep counts differ by step {100 * (chunk + 1)}"
        print(f"step {100 * (chunk + 1)}", flush=True)
    errs = compare(g, o)
    print({k: f"{v:.2e}" for k, v in errs.items()})
    dg, do = g.diag(), o.diag()
    for k in ("sum_psi", "sum_f", "sum_g", "V_l", "V_s"):
        assert dg[k] == pytest.approx(do[k], rel=1e-12), k
    for k in ("front_y", "height", "max_u"):
        assert dg[k] == pytest.approx(do[k], rel=1e-9, abs=1e-14), k
    assert dg["V_s"] > 10  # the drop is freezing


@pytest.mark.parametrize("shape", [(0, 0), (16, 8)], ids=["default", "m16"])
@pytest.mark.parametrize("nx,ny", [(100, 37), (70, 45), (64, 3), (2, 16)])
def test_ragged_and_degenerate_grids(nx, ny, shape):
    """Grids that leave partial tiles (x not a multiple of 64, y not of 4), the smallest
    height the walls allow (ny = 3) and the narrowest periodic width (nx = 2), with the default
    sweep shape and with 16-sweep launches (a 64 x 64 region writing 32 x 32: the x wrap and
    the walls fall inside one region)."""
    if nx >= 32 and ny >= 16:
        c = inputs.sessile_drop(nx, ny, min(nx, ny) / 3, 60.0, 3.0, 1.0, 0.2, 0.2, seed=7)
    else:
        c = inputs.stefan_strip(nx, ny, h0=ny / 2, Ste=0.2, rho_ratio_sl=0.9)
        inputs.set_electric(c, 2.0, 3.0, 0.0, 1.0)
    c.update(poisson_tol=1e-10)
    g, o = solver(dict(c, sweep_block=shape[0], sweep_waves=shape[1])), ob.Oracle(c)
    g.step(25)
    o.step(25)
    assert list(g.sweep_log()) == list(o.sweep_log())
    compare(g, o)


@pytest.mark.parametrize("ratio,theta", [(0.9, 120.0), (1.1, 45.0), (1.0, 90.0)])
def test_contact_angles_and_volume_change(ratio, theta):
    c = inputs.sessile_drop(96, 48, 16, theta, 2.0, 5.0, 1.0, 0.2, seed=3, rho_ratio_sl=ratio)
    g, o = solver(c), ob.Oracle(c)
    g.step(40)
    o.step(40)
    assert list(g.sweep_log()) == list(o.sweep_log())
    compare(g, o)


def test_without_grad_s_reading():
    c = small_drop(2)
    c["readings"] = 0
    g, o = solver(c), ob.Oracle(c)
    g.step(10)
    o.step(10)
    compare(g, o)


def test_set_state_then_step():
    """Inject a state into both sides (set_field / set_pop) and step: the library honours
    externally supplied fields and populations."""
    c = small_drop(0, 64, 32)
    g, o = solver(c), ob.Oracle(c)
    o.step(5)
    for k in ("psi", "ux", "uy", "usx", "usy", "p", "T", "H", "fs", "mdot", "psiu_x", "psiu_y"):
        g.set_field(k, o.field(k))
    for k in ("f", "h", "g"):
        g.set_pop(k, o.pop(k))
    g.set_pop("l", o.pop("l")[1:])
    g.set_field("phi", o.field("phi"))
    g.step(3)
    o.step(3)
    compare(g, o)


def test_diagnostics_and_freezing_time():
    """Strip freezing to completion: on-device FP64 freezing-time detector against the
    oracle's."""
    c = inputs.stefan_strip(4, 32, h0=10.0, Ste=0.5, rho_ratio_sl=0.9)
    g, o = solver(c), ob.Oracle(c)
    for _ in range(12):
        g.step(200)
        o.step(200)
    dg, do = g.diag(), o.diag()
    assert do["t_fre"] > 0
    assert dg["t_fre"] == pytest.approx(do["t_fre"], rel=1e-9)
    for k in ("V_l", "V_s", "sum_psi", "V_l0"):
        assert dg[k] == pytest.approx(do[k], rel=1e-11, abs=1e-13), k


def test_error_paths():
    from paper_2410_06657_amd import lbm
    c = small_drop(0, 64, 32)
    bad = dict(c, mu_l=-1.0)
    with pytest.raises(lbm.LbmError) as e:
        lbm.Solver(bad)
    assert e.value.code == lbm.LBM_EINVAL
    g = solver(c)
    rc, k, r = g.solve_potential(1e-300, 2)
    assert rc == lbm.LBM_ENOCONV and k == 2
    psi = g.field("psi")
    psi[3, 3] = np.nan
    g.set_field("psi", psi)
    d = g.diag()
    assert d["nonfinite"] == 1


def test_full_size_sampled():
    """The 4096 x 2048 workload in the benchmark's launch configuration: initialise and run
    two steps with a fixed sweep count on both sides, compare every field."""
    c = inputs.drop_4096x2048()
    c.update(poisson_tol=-1.0, poisson_max_sweeps=8)
    g = solver(c)
    o = ob.Oracle(c)
    g.step(2)
    o.step(2)
    compare(g, o, fields=["psi", "ux", "uy", "p", "T", "H", "fs", "phi"], pops=False)


def test_sweep_block_invariance():
    """Every launch shape (sweeps per launch x waves per workgroup) gives bitwise the same
    state (the per-node arithmetic of a sweep does not depend on the blocking) and the same
    sweep counts as the oracle."""
    c = small_drop(1, 96, 48)
    o = ob.Oracle(c)
    o.step(12)
    ref = None
    for m, w in ((1, 4), (2, 4), (4, 4), (8, 4), (1, 8), (2, 8), (4, 8), (8, 8), (16, 8)):
        g = solver(dict(c, sweep_block=m, sweep_waves=w))
        g.step(12)
        assert list(g.sweep_log()) == list(o.sweep_log()), (m, w)
        state = {k: g.field(k) for k in ("psi", "ux", "uy", "p", "T", "phi")}
        state["l"] = g.pop("l")
        if ref is None:
            ref = state
            compare(g, o)
        else:
            for k in state:
                assert np.array_equal(state[k], ref[k]), (m, w, k)


@pytest.mark.parametrize("m", [1, 8, 16])
def test_checkerboard_link_sum_alternates_on_the_gpu(m):
    """The sweep kernel keeps the D2Q5 scheme's undamped mode as the oracle does (its pin is in
    test_oracle_potential.py): from random links, the checkerboard sum of the four moving links
    changes sign exactly, sweep after sweep, in launches of one and of eight sweeps, and the
    links after 8 sweeps equal the oracle's."""
    c = small_drop(2, 96, 48)
    c.update(poisson_tol=-1.0, poisson_max_sweeps=2)
    g, o = solver(dict(c, sweep_block=m, sweep_waves=8 if m == 16 else 0)), ob.Oracle(c)
    rng = np.random.default_rng(7)
    links = o.pop("l") + 1e-3 * rng.normal(size=(5, 48, 96))
    o.set_pop("l", links)
    g.set_pop("l", links[1:])
    chk = (-1.0) ** (np.arange(48)[:, None] + np.arange(96)[None, :])
    q = float((chk * g.pop("l").sum(axis=0)).sum())
    scale = float(np.abs(links[1:]).sum())
    assert abs(q) > 1e-5 * scale
    for k in range(8):
        g.solve_potential(-1.0, 1)
        q1 = float((chk * g.pop("l").sum(axis=0)).sum())
        assert abs(q1 + q) <= 1e-13 * scale, (k, q, q1)
        q = q1
    o.solve_potential(-1.0, 8)
    assert np.allclose(g.pop("l"), o.pop("l")[1:], rtol=0, atol=1e-13)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_checkpoint_restore_continues_bitwise(precision):
    """A checkpoint taken mid-run, restored into a fresh handle of the same case, continues
    bitwise as the original run (fields, populations, sweep log, freezing detector)."""
    from paper_2410_06657_amd.lbm import LbmError, Solver, LBM_EINVAL
    c = small_drop(4, 96, 48)
    a = Solver(c, precision)
    a.step(15)
    img = a.checkpoint()
    a.step(10)
    b = Solver(c, precision)
    b.restore(img)
    b.step(10)
    assert list(a.sweep_log()) == list(b.sweep_log())
    for k in FIELDS:
        assert np.array_equal(a.field(k), b.field(k)), k
    for k in ("f", "h", "g", "l"):
        assert np.array_equal(a.pop(k), b.pop(k)), k
    da, db = a.diag(), b.diag()
    assert da["step"] == db["step"] == 25 and da["V_s"] == db["V_s"]
    # an image of another grid is refused
    other = Solver(small_drop(4, 64, 32), precision)
    with pytest.raises(LbmError) as e:
        other.restore(img)
    assert e.value.code == LBM_EINVAL
