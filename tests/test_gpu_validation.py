"""The paper's validation problems on the GPU path: the deformation of a free drop in a
uniform field against the small-deformation theories (Sec. 4, Fig. 5), and the three-phase
Stefan problem (Sec. 4, Fig. 2): the one-phase Neumann front and the final height of a layer
freezing with volume change.  The geometries first match the FP64 oracle element by element
(1e-10), then the sweeps run as FP64 batches (one launch per stage for all cases)."""
import math
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu

# Fig. 5: (a) R = 5 with S swept, (b) S = 2 with R swept, Ca_E = 0.2 in both
CA_E = 0.2
S_SWEEP = [(5.0, S) for S in (1.0, 3.0, 6.0, 9.0, 12.0, 15.0)]
R_SWEEP = [(R, 2.0) for R in (0.5, 1.0, 2.0, 3.0, 5.0, 8.0)]


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    ob.set_threads(min(16, os.cpu_count() or 1))
    yield
    ob.set_threads(1)


def rel_l2(a, b):
    den = max(np.linalg.norm(b), 1e-12 * math.sqrt(np.asarray(b).size))
    return float(np.linalg.norm(np.asarray(a) - b) / den)


def feng(R, S, Ca):
    """2D first-order deformation (Feng), D = (L - H) / (L + H) with L along the field."""
    return Ca * (R * R + R + 1 - 3 * S) / (3 * (1 + R) ** 2)


def taylor(R, S, Ca, B=1.0):
    """Taylor's 3D small-deformation value, f_T as printed in Sec. 4 (viscosity ratio B)."""
    fT = R * R + 1 - 2 * S + 0.6 * (R - S) * (2 + 3 * B) / (1 + B)
    return 9 * Ca / 16 * fT / (2 + R) ** 2


def deformation(psi, c):
    """(L - H)/(L + H) from the psi = 1/2 crossings through the drop centre (L: along y)."""
    ic, jc = int(round(c["xc"])), int(round(c["yc"]))

    def span(v):
        idx = np.where(v >= 0.5)[0]
        a, b = idx[0], idx[-1]
        lo = a - (v[a] - 0.5) / (v[a] - v[a - 1])
        hi = b + (v[b] - 0.5) / (v[b] - v[b + 1])
        return hi - lo

    L, H = span(psi[:, ic]), span(psi[jc, :])
    return (L - H) / (L + H)


@pytest.mark.parametrize("case,steps", [
    (inputs.free_drop(64, 64, 10.0, R=5.0, S=2.0, Ca_E=CA_E), 40),
    (inputs.stefan_strip(4, 48, h0=16.0, Ste=0.5, rho_ratio_sl=0.9), 400),
], ids=["free_drop", "stefan_strip"])
def test_validation_geometries_match_oracle(case, steps):
    """Element-wise FP64 parity.  The free drop is held for 40 steps: its spurious interface
    currents are chaotic, so the method itself, restarted from populations perturbed by 1e-15
    (relative), departs from the unperturbed run by 1e-7 to 1e-3 after 100-150 steps (measured
    on the GPU; the sessile 128 x 64 drop stays within 1e-11 over 1000 steps).  The strip is
    held for 400 steps."""
    from paper_2410_06657_amd.lbm import Solver
    g, o = Solver(case), ob.Oracle(case)
    g.step(steps)
    o.step(steps)
    assert list(g.sweep_log()) == list(o.sweep_log())
    errs = {k: rel_l2(g.field(k), o.field(k)) for k in ("psi", "ux", "uy", "p", "T", "fs", "phi")}
    print({k: f"{v:.1e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-10, errs


def test_free_drop_deformation_sweep():
    """Fig. 5's two sweeps as one batch of 12 drops (R0 = 20 in 160 x 160).  D is read every
    1,000 steps from 6,000 to 10,000 (the shapes have settled; D oscillates by about 1e-3) and
    averaged.  Every point has Feng's sign and lies between the Taylor and Feng values within
    15% of the larger of them plus 0.003 (measured: all inside the band but R = 0.5 and S = 9,
    11% and 0.0014 beyond Feng), D falls with S and rises with R, and the change from prolate
    to oblate sits where Feng's f_F = R^2 + R + 1 - 3S changes sign."""
    from paper_2410_06657_amd.lbm import Batch
    pts = S_SWEEP + R_SWEEP
    cases = [inputs.free_drop(160, 160, 20.0, R=R, S=S, Ca_E=CA_E) for R, S in pts]
    b = Batch(cases, precision="fp64")
    b.step(5000)
    samples = []
    for _ in range(5):
        b.step(1000)
        samples.append([deformation(b.field(k, "psi"), cases[k]) for k in range(len(pts))])
    samples = np.array(samples)
    D = samples.mean(axis=0)
    for k, (R, S) in enumerate(pts):
        x, f, t = D[k], feng(R, S, CA_E), taylor(R, S, CA_E)
        spread = samples[:, k].max() - samples[:, k].min()
        print(f"R={R} S={S}: D {x:+.4f} (spread {spread:.4f}), Feng {f:+.4f}, Taylor {t:+.4f}")
        assert spread <= 0.003
        assert np.sign(x) == np.sign(f)
        tol = 0.15 * max(abs(f), abs(t)) + 0.003
        assert min(f, t) - tol <= x <= max(f, t) + tol
    ds, dr = D[:len(S_SWEEP)], D[len(S_SWEEP):]
    assert all(p > q for p, q in zip(ds, ds[1:]))
    assert all(p < q for p, q in zip(dr, dr[1:]))


def test_neumann_front_sweep():
    """One-phase Stefan problem (liquid at T_m, substrate at -Ste, alpha_s = 0.2): the f_l = 1/2
    front follows s = 2 lambda sqrt(alpha_s t) within 2% for Ste = 0.05, 0.1, 0.2, 0.5, read
    when the front has travelled about 12, 18 and 24 nodes."""
    from paper_2410_06657_amd.lbm import Batch
    stes = (0.05, 0.1, 0.2, 0.5)
    alpha = 0.2
    cases = [inputs.stefan_strip(4, 48, h0=1e6, Ste=s, rho_ratio_sl=1.0, alpha_s=alpha) for s in stes]
    b = Batch(cases, precision="fp64")
    lams = [neumann_lambda(s) for s in stes]
    chunk = 250
    when = [{chunk * math.ceil((x / (2 * lam)) ** 2 / alpha / chunk) for x in (12.0, 18.0, 24.0)} for lam in lams]
    errs = [[] for _ in stes]
    t = 0
    while t < max(max(w) for w in when):
        b.step(chunk)
        t += chunk
        for k, lam in enumerate(lams):
            if t not in when[k]:
                continue
            fl = b.field(k, "fl")[:, 0]
            m = np.where(fl >= 0.5)[0][0]
            s = (m - 1) + (0.5 - fl[m - 1]) / (fl[m] - fl[m - 1]) + 0.5
            ref = 2 * lam * math.sqrt(alpha * t)
            errs[k].append(abs(s - ref) / ref)
    for ste, e in zip(stes, errs):
        print(f"Ste={ste}: front errors {[f'{x:.4f}' for x in e]}")
        assert len(e) == 3
    assert max(max(e) for e in errs) < 0.02


def neumann_lambda(ste):
    """Root of lambda exp(lambda^2) erf(lambda) = Ste / sqrt(pi) (one-phase Neumann)."""
    lo, hi = 1e-9, 2.0
    f = lambda x: x * math.exp(x * x) * math.erf(x) - ste / math.sqrt(math.pi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def test_final_height_sweep():
    """Layers of h0 = 16 freezing completely at Ste = 0.2, 0.5 with rho_s/rho_l = 0.9, 1.0,
    1.1: the material volume ends at rho_l/rho_s of its start (h_f = rho_l h_0 / rho_s) within 1%."""
    from paper_2410_06657_amd.lbm import Batch
    grid = [(s, r) for s in (0.2, 0.5) for r in (0.9, 1.0, 1.1)]
    cases = [inputs.stefan_strip(4, 48, h0=16.0, Ste=s, rho_ratio_sl=r) for s, r in grid]
    b = Batch(cases, precision="fp64")
    v0 = [b.field(k, "psi").clip(0, 1).sum() / 4 for k in range(len(grid))]
    for _ in range(60):
        b.step(500)
        if all(d["V_l"] < 1e-4 * d["V_l0"] for d in b.diag()):
            break
    ds = b.diag()
    for k, (s, r) in enumerate(grid):
        v1 = b.field(k, "psi").clip(0, 1).sum() / 4
        print(f"Ste={s} rho_s/rho_l={r}: V_l/V_l0 {ds[k]['V_l'] / ds[k]['V_l0']:.1e}, "
              f"h_f/h_0 {v1 / v0[k]:.4f} (closed form {1 / r:.4f})")
        assert ds[k]["V_l"] < 1e-3 * ds[k]["V_l0"], "layer did not freeze"
        assert v1 / v0[k] == pytest.approx(1 / r, rel=0.01)
