"""The paper's validation problems on the GPU path (runners in
paper_2410_06657_amd/validation.py): the deformation of a free drop in a uniform field against
the small-deformation theories (Sec. 4, Fig. 5), and the three-phase Stefan problem (Sec. 4,
Fig. 2): the one-phase Neumann front and the final height of a layer freezing with volume
change.  The two geometries first match the FP64 oracle element by element (1e-10); the sweeps
then run as FP64 batches (one launch per stage for all cases)."""
import math
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs, validation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    ob.set_threads(min(16, os.cpu_count() or 1))
    yield
    ob.set_threads(1)


def rel_l2(a, b):
    den = max(np.linalg.norm(b), 1e-12 * math.sqrt(np.asarray(b).size))
    return float(np.linalg.norm(np.asarray(a) - b) / den)


@pytest.mark.parametrize("case,steps", [
    (inputs.free_drop(64, 64, 10.0, R=5.0, S=2.0, Ca_E=validation.CA_E), 40),
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
    res = validation.deformation_sweep()
    for r in res:
        x, f, t = r["D"], r["feng"], r["taylor"]
        print(f"R={r['R']} S={r['S']}: D {x:+.4f} (spread {r['spread']:.4f}), Feng {f:+.4f}, Taylor {t:+.4f}")
        assert r["spread"] <= 0.003
        assert np.sign(x) == np.sign(f)
        tol = 0.15 * max(abs(f), abs(t)) + 0.003
        assert min(f, t) - tol <= x <= max(f, t) + tol
    n = len(validation.S_SWEEP)
    ds, dr = [r["D"] for r in res[:n]], [r["D"] for r in res[n:]]
    assert all(p > q for p, q in zip(ds, ds[1:]))
    assert all(p < q for p, q in zip(dr, dr[1:]))


def test_neumann_front_sweep():
    """One-phase Stefan problem (liquid at T_m, substrate at -Ste, alpha_s = 0.2): the f_l = 1/2
    front follows s = 2 lambda sqrt(alpha_s t) within 2% for Ste = 0.05, 0.1, 0.2, 0.5, read
    when the front has travelled about 12, 18 and 24 nodes."""
    res = validation.neumann_sweep()
    for r in res:
        print(f"Ste={r['Ste']}: front errors {[f'{x:.4f}' for x in r['rel_err']]}")
        assert len(r["rel_err"]) == 3
        assert max(r["rel_err"]) < 0.02


def test_final_height_sweep():
    """Layers of h0 = 16 freezing completely at Ste = 0.2, 0.5 with rho_s/rho_l = 0.9, 1.0,
    1.1: the material volume ends at rho_l/rho_s of its start (h_f = rho_l h_0 / rho_s) within 1%."""
    for r in validation.final_height_sweep():
        print(f"Ste={r['Ste']} rho_s/rho_l={r['rho_s_over_rho_l']}: liquid left {r['liquid_left']:.1e}, "
              f"h_f/h_0 {r['h_f_over_h_0']:.4f} (closed form {r['closed_form']:.4f})")
        assert r["liquid_left"] < 1e-3, "layer did not freeze"
        assert r["h_f_over_h_0"] == pytest.approx(r["closed_form"], rel=0.01)


def test_parameter_study():
    """Sec. 5 at theta = 120 deg: no field, PR+ (2, 0.5), OB- (2, 5), PR- (5, 9.5) with Ca_E = 1,
    Ste = 0.05, 0.1, 0.2, rho_s/rho_l = 0.9 and 1.1, each drop run to its freezing time.  What
    the paper reports and this checks: the substrate heat flux diminishes as the drop freezes
    and is lower at a smaller Stefan number; without a field the drop ends taller than it started
    when the solid is lighter and shorter when it is denser; the field makes the prolate PR+
    drop end taller and the oblate drop shorter than without it; the oblate drop freezes
    faster (t* < 0), by less as Ste grows, and the PR- drop slower (t* > 0).  Measured beside
    it (not asserted): the PR+ time change is within 0.2% for rho_s/rho_l = 0.9."""
    rows = validation.parameter_study()
    by = {(x["rho_s_over_rho_l"], x["Ste"], x["mode"]): x for x in rows}
    # the heat flux into the substrate falls as the drop freezes, and starts higher at a larger
    # Stefan number (measured 0.0020 / 0.0028 / 0.0040 at Fo = 0.25 for Ste = 0.05 / 0.1 / 0.2)
    for x in rows:
        q = [v for _, v in x["substrate_flux"]]
        assert len(q) >= 2 and all(b <= a + 1e-12 for a, b in zip(q, q[1:])), (x["Ste"], x["mode"], q)
    for r in (0.9, 1.1):
        for m in validation.MODES:
            q0 = [by[(r, s, m)]["substrate_flux"][0][1] for s in (0.05, 0.1, 0.2)]
            assert q0[0] < q0[1] < q0[2], (r, m, q0)
    # H_m / R_0 ~ (Ste Fo)^(1/2): the coefficient varies by at most 1.8x over the 24 cases
    # (measured 1.65x; 1.25x and 1.39x within each density ratio).  Ste Fo spans only 0.19-0.29
    # here, so the exponent itself is not tested.
    law = validation.ste_fo_law(rows)
    print("Ste Fo law", law)
    assert law["coefficient_spread"] <= 1.8
    for x in rows:
        print(f"rho {x['rho_s_over_rho_l']} Ste {x['Ste']} {x['mode']:>4}: t_fre {x['t_fre']:.0f} "
              f"Fo {x['Fo']:.3f} H_m/H_0 {x['H_m_over_H_0']:.4f} t* {x['t_star']:+.4f}")
    for r in (0.9, 1.1):
        ob_mag = []
        for s in (0.05, 0.1, 0.2):
            h = {m: by[(r, s, m)]["H_m_over_H_0"] for m in validation.MODES}
            assert (h["none"] > 1.0) if r < 1 else (h["none"] < 1.0)
            assert h["PR+"] > h["none"] > h["OB-"]
            assert by[(r, s, "OB-")]["t_star"] < 0
            assert by[(r, s, "PR-")]["t_star"] > 0
            ob_mag.append(-by[(r, s, "OB-")]["t_star"])
        assert ob_mag[0] > ob_mag[-1]


def test_cold_wall_freezing():
    """Sec. 4's drop freezing on a cold wall with Table 1's ratios (theta = 87 deg; water:
    Ste = 0.127, rho_s/rho_l = 0.918, k_s/k_l = 3.72; hexadecane: Ste = 0.030, rho_s/rho_l =
    1.076), each frozen completely.  The material volume ends at rho_l/rho_s of its start within
    1.5% (measured -1.1% and +0.7%); the water drop ends taller with a sharper apex (the tip the
    paper describes) and the hexadecane drop shorter with a flatter top (its platform)."""
    res = {r["liquid"]: r for r in validation.cold_wall()}
    for r in res.values():
        print({k: (round(float(x), 4) if isinstance(x, float) else x) for k, x in r.items()})
        assert r["volume_ratio"] == pytest.approx(r["closed_form_volume_ratio"], rel=0.015)
    w, h = res["water"], res["hexadecane"]
    assert w["H_m_over_H_0"] > 1.05 and h["H_m_over_H_0"] < 0.95
    assert abs(w["apex_curvature"]) > 1.15 * abs(w["apex_curvature_start"])
    assert abs(h["apex_curvature"]) < abs(h["apex_curvature_start"])
