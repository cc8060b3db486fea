"""The stored one-rounding drift envelope (tests/golden/fp32_envelope_128x64.txt) is the
oracle's own: the first checkpoints of injection seed 1, recomputed here, match the stored
rows, and every 'max' row is the largest of the seed rows at its step."""
import importlib.util
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def generator():
    spec = importlib.util.spec_from_file_location("make_fp32_envelope",
                                                  os.path.join(GOLDEN, "make_fp32_envelope.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def stored():
    rows = {}
    with open(os.path.join(GOLDEN, "fp32_envelope_128x64.txt")) as f:
        for line in f:
            p = line.split()
            if p and (p[0] == "max" or p[0].startswith("seed")):
                rows[(p[0], int(p[1]))] = np.array([float(v) for v in p[2:]])
    return rows


def test_max_rows_are_the_seed_maxima():
    rows = stored()
    steps = sorted({n for k, n in rows if k == "max"})
    seeds = sorted({k for k, n in rows if k.startswith("seed")})
    assert len(seeds) >= 3 and 1000 in steps
    for n in steps:
        assert np.array_equal(rows[("max", n)], np.max([rows[(s, n)] for s in seeds], axis=0)), n


def test_seed1_rows_reproduce():
    gen = generator()
    ob.set_threads(min(8, os.cpu_count() or 1))
    try:
        got = gen.drift(inputs.drop_128x64(0), 1, steps=20)
    finally:
        ob.set_threads(1)
    rows = stored()
    for n in (10, 20):
        want = rows[("seed1", n)]
        vals = np.array([got[n][k] for k in gen.FIELDS])
        assert vals == pytest.approx(want, rel=1e-5), n
