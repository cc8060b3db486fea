"""Writes fp32_envelope_128x64.txt: how far the FP64 oracle drifts from itself on the 128 x 64
sessile drop (R0 = 24, theta = 90, R = 3, S = 1, Ca_E = 0.1, Ste = 0.1, seed 0) when every step
leaves a single-precision rounding error on the state, the error a single-precision form
cannot avoid.  After each step every f, h and g population and every potential link is
multiplied by 1 + 2^-24 u with u uniform on [-1, 1] (SplitMix64-seeded numpy generator), the
relative size of one FP32 rounding; the relative L2 difference per field from the
unperturbed oracle is recorded at fixed steps, and the envelope is the largest over several
injection seeds.  Calls only the oracle.  Run: python tests/golden/make_fp32_envelope.py"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.binding import Oracle, set_threads  # noqa: E402
from paper_2410_06657_amd import inputs  # noqa: E402

FIELDS = ["psi", "ux", "uy", "p", "T", "H", "fs", "phi"]
CHECKPOINTS = (10, 20, 50, 100, 200, 300, 400, 500, 600, 700, 800, 900, 1000)
OUT = os.path.join(HERE, "fp32_envelope_128x64.txt")


def rel_l2(a, b):
    den = max(np.linalg.norm(b), 1e-12 * np.sqrt(b.size))
    return float(np.linalg.norm(a - b) / den)


def perturb(o, rng):
    for k in ("f", "h", "g", "l"):
        p = o.pop(k)
        o.set_pop(k, p * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, p.shape)))


def drift(case, seed, steps=max(CHECKPOINTS)):
    """Per-field relative L2 distance of the perturbed run from the plain run at each
    checkpoint."""
    a, b = Oracle(case), Oracle(case)
    rng = np.random.default_rng(seed)
    rows = {}
    for n in range(1, steps + 1):
        a.step(1)
        b.step(1)
        perturb(b, rng)
        if n in CHECKPOINTS:
            rows[n] = {k: rel_l2(b.field(k), a.field(k)) for k in FIELDS}
            print(f"seed {seed} step {n}: max {max(rows[n].values()):.3e}", flush=True)
    return rows


def main(seeds=(1, 2, 3, 4)):
    set_threads(min(8, os.cpu_count() or 1))
    case = inputs.drop_128x64(0)
    runs = [drift(case, s) for s in seeds]
    with open(OUT, "w") as f:
        f.write("# FP64 oracle with one FP32 rounding (relative 2^-24, uniform) injected into every f, h, g\n")
        f.write("# population and potential link after every step; relative L2 distance per field from the\n")
        f.write("# plain oracle, largest over injection seeds " + " ".join(map(str, seeds)) + ".\n")
        f.write("# case: 128x64 sessile drop, R0=24, theta=90, R=3, S=1, Ca_E=0.1, Ste=0.1, seed 0\n")
        f.write("# written by tests/golden/make_fp32_envelope.py (oracle only)\n")
        f.write("# rows: 'max' (largest over the seeds) or 'seed <s>', then the step and one value per field\n")
        f.write("kind step " + " ".join(FIELDS) + "\n")
        for n in CHECKPOINTS:
            vals = [max(r[n][k] for r in runs) for k in FIELDS]
            f.write(f"max {n} " + " ".join(f"{v:.6e}" for v in vals) + "\n")
        for sd, r in zip(seeds, runs):
            for n in CHECKPOINTS:
                f.write(f"seed{sd} {n} " + " ".join(f"{r[n][k]:.6e}" for k in FIELDS) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
