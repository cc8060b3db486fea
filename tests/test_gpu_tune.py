"""Autotuner of the potential-sweep launch shape: it picks one of the timed candidates, a
repeated call is served from the cache, and a solver run with the chosen shape equals the
default-shape run bitwise (the shape changes speed only)."""
import numpy as np
import pytest

from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_choice_cache_and_invariance(precision, tmp_path, monkeypatch):
    from paper_2410_06657_amd import lbm
    monkeypatch.setenv("LBM_TUNE_CACHE", str(tmp_path / "shapes.json"))
    c = inputs.scaled(inputs.drop_128x64(3), 256, 128)
    r = lbm.autotune(c, precision, launches=10, force=True)
    print(r)
    cands = {(k["sweep_block"], k["sweep_waves"]): k["us_per_sweep"] for k in r["candidates"]}
    assert len(cands) == 6 and all(v > 0 for v in cands.values())
    best = (r["sweep_block"], r["sweep_waves"])
    assert cands[best] == min(cands.values())
    again = lbm.autotune(c, precision, launches=10)
    assert again["cached"] == "file" and (again["sweep_block"], again["sweep_waves"]) == best
    lib_cached = lbm.autotune(c, precision, launches=10, persist=False)
    assert lib_cached["cached"] == "library"
    assert (lib_cached["sweep_block"], lib_cached["sweep_waves"]) == best
    a = lbm.Solver(c, precision)
    b = lbm.Solver(dict(c, sweep_block=best[0], sweep_waves=best[1]), precision)
    a.step(6)
    b.step(6)
    assert list(a.sweep_log()) == list(b.sweep_log())
    for k in ("psi", "ux", "p", "T", "phi"):
        assert np.array_equal(a.field(k), b.field(k)), k
