"""The paper's validation problems (Sec. 4) run on the library, each sweep as one batch.

* Deformation of a free leaky-dielectric drop in a uniform field (Fig. 5): D = (L - H)/(L + H),
  L the extent along the field, against Taylor's small-deformation value (f_T as printed in
  Sec. 4) and Feng's 2D first-order value; R = 5 with S swept and S = 2 with R swept, Ca_E = 0.2.
* Three-phase Stefan problem (Fig. 2): the one-phase Neumann front s = 2 lambda sqrt(alpha_s t)
  of a liquid at T_m on a substrate at -Ste, and the final height h_f = rho_l h_0 / rho_s of a
  layer that freezes completely.

* Freezing of water and hexadecane drops on a cold wall with Table 1's property ratios (Sec. 4):
  final volume against rho_l/rho_s, height, contact radius and apex shape.
* The electrofreezing study of Sec. 5: a wetting drop (theta = 120 deg) frozen without a field
  and in the PR+, OB- and PR- modes of its R-S diagram at several Stefan numbers and
  solid/liquid density ratios: final heights, the relative change of the freezing time, the
  heat flux into the substrate over time, and the H_m/R_0 ~ (Ste Fo)^(1/2) law of Sec. 5.

Freezing is off for the free drops (T_w = T_g above T_m).  Inputs come from
`inputs.free_drop`, `inputs.stefan_strip` and `inputs.sessile_drop`.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs

CA_E = 0.2
S_SWEEP = [(5.0, S) for S in (1.0, 3.0, 6.0, 9.0, 12.0, 15.0)]   # Fig. 5(a): R = 5
R_SWEEP = [(R, 2.0) for R in (0.5, 1.0, 2.0, 3.0, 5.0, 8.0)]     # Fig. 5(b): S = 2


def feng(R: float, S: float, Ca: float) -> float:
    """Feng's 2D first-order deformation, D = Ca_E f_F / (3 (1 + R)^2), f_F = R^2 + R + 1 - 3S."""
    return Ca * (R * R + R + 1 - 3 * S) / (3 * (1 + R) ** 2)


def taylor(R: float, S: float, Ca: float, B: float = 1.0) -> float:
    """Taylor's small-deformation value 9 Ca_E f_T / (16 (2 + R)^2), B the viscosity ratio."""
    fT = R * R + 1 - 2 * S + 0.6 * (R - S) * (2 + 3 * B) / (1 + B)
    return 9 * Ca / 16 * fT / (2 + R) ** 2


def neumann_lambda(ste: float) -> float:
    """Root of lambda exp(lambda^2) erf(lambda) = Ste / sqrt(pi) (one-phase Neumann problem)."""
    lo, hi = 1e-12, 3.0
    f = lambda x: x * math.exp(x * x) * math.erf(x) - ste / math.sqrt(math.pi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def _span(v: np.ndarray) -> float:
    """Length of the psi >= 1/2 run along a line, ends interpolated linearly."""
    idx = np.where(v >= 0.5)[0]
    a, b = idx[0], idx[-1]
    lo = a - (v[a] - 0.5) / (v[a] - v[a - 1])
    hi = b + (v[b] - 0.5) / (v[b] - v[b + 1])
    return hi - lo


def deformation(psi: np.ndarray, case: dict) -> float:
    """(L - H)/(L + H) through the drop centre; the field is along y."""
    ic, jc = int(round(case["xc"])), int(round(case["yc"]))
    L, H = _span(psi[:, ic]), _span(psi[jc, :])
    return (L - H) / (L + H)


def front(fl_column: np.ndarray) -> float:
    """Distance of the f_l = 1/2 crossing from the substrate (the wall is at y = -1/2)."""
    m = int(np.where(fl_column >= 0.5)[0][0])
    return (m - 1) + (0.5 - fl_column[m - 1]) / (fl_column[m] - fl_column[m - 1]) + 0.5


def deformation_sweep(n: int = 160, R0: float = 20.0, settle: int = 5000, samples: int = 5,
                      every: int = 1000, precision: str = "fp64") -> list[dict]:
    """Both Fig. 5 sweeps as one batch; D averaged over `samples` readings `every` steps apart
    after `settle` steps."""
    from .lbm import Batch
    pts = S_SWEEP + R_SWEEP
    cases = [inputs.free_drop(n, n, R0, R=R, S=S, Ca_E=CA_E) for R, S in pts]
    b = Batch(cases, precision=precision)
    b.step(settle)
    reads = []
    for _ in range(samples):
        b.step(every)
        reads.append([deformation(b.field(k, "psi"), cases[k]) for k in range(len(pts))])
    reads = np.array(reads)
    out = []
    for k, (R, S) in enumerate(pts):
        out.append({"R": R, "S": S, "D": float(reads[:, k].mean()),
                    "spread": float(reads[:, k].max() - reads[:, k].min()),
                    "feng": feng(R, S, CA_E), "taylor": taylor(R, S, CA_E)})
    return out


def neumann_sweep(stes=(0.05, 0.1, 0.2, 0.5), alpha: float = 0.2, ny: int = 48,
                  at=(12.0, 18.0, 24.0), chunk: int = 250, precision: str = "fp64") -> list[dict]:
    """Front position against Neumann's when the front has travelled about `at` nodes."""
    from .lbm import Batch
    cases = [inputs.stefan_strip(4, ny, h0=1e6, Ste=s, rho_ratio_sl=1.0, alpha_s=alpha) for s in stes]
    b = Batch(cases, precision=precision)
    lams = [neumann_lambda(s) for s in stes]
    when = [sorted({chunk * math.ceil((x / (2 * lam)) ** 2 / alpha / chunk) for x in at}) for lam in lams]
    res = [{"Ste": s, "lambda": lam, "t": [], "s": [], "s_neumann": [], "rel_err": []}
           for s, lam in zip(stes, lams)]
    t = 0
    while t < max(w[-1] for w in when):
        b.step(chunk)
        t += chunk
        for k, lam in enumerate(lams):
            if t in when[k]:
                s = front(b.field(k, "fl")[:, 0])
                ref = 2 * lam * math.sqrt(alpha * t)
                r = res[k]
                r["t"].append(t)
                r["s"].append(s)
                r["s_neumann"].append(ref)
                r["rel_err"].append(abs(s - ref) / ref)
    return res


def final_height_sweep(stes=(0.2, 0.5), ratios=(0.9, 1.0, 1.1), h0: float = 16.0, ny: int = 48,
                       chunk: int = 500, max_chunks: int = 60, precision: str = "fp64") -> list[dict]:
    """Layers freezing completely; the material volume per column ends at rho_l/rho_s of its
    start (h_f / h_0 = rho_l / rho_s)."""
    from .lbm import Batch
    grid = [(s, r) for s in stes for r in ratios]
    cases = [inputs.stefan_strip(4, ny, h0=h0, Ste=s, rho_ratio_sl=r) for s, r in grid]
    b = Batch(cases, precision=precision)
    v0 = [b.field(k, "psi").clip(0, 1).sum() / 4 for k in range(len(grid))]
    steps = 0
    for _ in range(max_chunks):
        b.step(chunk)
        steps += chunk
        if all(d["V_l"] < 1e-4 * d["V_l0"] for d in b.diag()):
            break
    ds = b.diag()
    out = []
    for k, (s, r) in enumerate(grid):
        v1 = b.field(k, "psi").clip(0, 1).sum() / 4
        out.append({"Ste": s, "rho_s_over_rho_l": r, "steps": steps,
                    "liquid_left": ds[k]["V_l"] / ds[k]["V_l0"],
                    "h_f_over_h_0": float(v1 / v0[k]), "closed_form": 1.0 / r})
    return out


# Sec. 5: field modes of the wetting drop (R, S, Ca_E); "none" is the drop without a field
MODES = {"none": (1.0, 1.0, 0.0), "PR+": (2.0, 0.5, 1.0), "OB-": (2.0, 5.0, 1.0), "PR-": (5.0, 9.5, 1.0)}


def drop_height(psi: np.ndarray, case: dict) -> float:
    """Height of the psi = 1/2 crossing on the drop's centre column above the substrate."""
    col = psi[:, int(round(case["xc"]))]
    b = int(np.where(col >= 0.5)[0][-1])
    return b + (col[b] - 0.5) / (col[b] - col[b + 1]) + 0.5


def substrate_heat_flux(T: np.ndarray, psi: np.ndarray, fs: np.ndarray, case: dict) -> np.ndarray:
    """Heat flux into the substrate along x, lambda dT/dy at the bottom row (Sec. 5: Fourier's
    law with the second-order one-sided difference (4 T_1 - T_2 - 3 T_0) / (2 dy) on the rows
    j = 0, 1, 2 above the wall, R31); lambda of the bottom row mixed by Eq. (1) with psi clamped.
    Positive when heat leaves the drop into the cold substrate (the paper's Qdot is its
    negative)."""
    pc = np.clip(psi[0], 0.0, 1.0)
    f = fs[0]
    lam = f * case["k_s"] + (1 - f) * pc * case["k_l"] + (1 - f) * (1 - pc) * case["k_g"]
    return lam * (4.0 * T[1] - T[2] - 3.0 * T[0]) / 2.0


def ste_fo_law(rows: list[dict]) -> dict:
    """Sec. 5's freezing-time law H_m / R_0 ~ (Ste Fo)^(1/2) over the study's cases: the slope
    of log(H_m/R_0) against log(Ste Fo) (least squares) and the spread of the coefficient
    (H_m/R_0) / (Ste Fo)^(1/2) (max over min)."""
    x = np.log([r["Ste"] * r["Fo"] for r in rows])
    y = np.log([r["H_m_over_R_0"] for r in rows])
    slope = float(np.polyfit(x, y, 1)[0])
    c = np.exp(y - 0.5 * x)
    return {"slope": slope, "coefficient_spread": float(c.max() / c.min()), "coefficient_mean": float(c.mean())}


def parameter_study(stes=(0.05, 0.1, 0.2), ratios=(0.9, 1.1), nx: int = 160, ny: int = 80,
                    R0: float = 20.0, theta: float = 120.0, precision: str = "fp64",
                    max_steps: int = 100000, sample_every: int = 1000) -> list[dict]:
    """Sec. 5's electrofreezing study at theta = 120 deg, alpha_l/alpha_g = 0.2: every field
    mode at every Stefan number and solid/liquid density ratio, run to its freezing time
    (1% of the liquid left) as one batch.  Per case: t_fre, Fo = alpha_l t_fre / R0^2, the final
    height H_m over the initial H_0 and over R_0, t* = (t_fre - t_fre(no field)) / t_fre(no
    field), and the mean heat flux into the substrate under the drop (contact region: bottom-row
    psi >= 1/2) every `sample_every` steps until the case freezes, as (Fo, flux) pairs."""
    from .lbm import Batch
    keys = [(r, s, m) for r in ratios for s in stes for m in MODES]
    cases = [inputs.sessile_drop(nx, ny, R0, theta, *MODES[m][:2], MODES[m][2], s, seed=None, rho_ratio_sl=r)
             for r, s, m in keys]
    b = Batch(cases, precision=precision)
    h0 = [drop_height(b.field(k, "psi"), cases[k]) for k in range(len(keys))]
    alpha = [c["k_l"] / (c["rho_l"] * c["cp_l"]) for c in cases]
    flux = [[] for _ in keys]
    done = 0
    while done < max_steps:
        n = b.run_until_frozen(min(sample_every, max_steps - done))
        done += n
        d = b.diag()
        for k in range(len(keys)):
            if flux[k] and flux[k][-1][0] == alpha[k] * d[k]["step"] / R0 ** 2:
                continue  # frozen: no new sample
            psi = b.field(k, "psi")
            q = substrate_heat_flux(b.field(k, "T"), psi, b.field(k, "fs"), cases[k])
            foot = psi[0] >= 0.5
            flux[k].append((alpha[k] * d[k]["step"] / R0 ** 2, float(q[foot].mean()) if foot.any() else 0.0))
        if n < sample_every:
            break
    d = b.diag()
    rows = []
    for k, (r, s, m) in enumerate(keys):
        hm = drop_height(b.field(k, "psi"), cases[k])
        rows.append({"rho_s_over_rho_l": r, "Ste": s, "mode": m, "t_fre": d[k]["t_fre"],
                     "Fo": alpha[k] * d[k]["t_fre"] / R0 ** 2,
                     "H_m_over_H_0": hm / h0[k], "H_m_over_R_0": hm / R0,
                     "substrate_flux": flux[k]})
    base = {(x["rho_s_over_rho_l"], x["Ste"]): x["t_fre"] for x in rows if x["mode"] == "none"}
    for x in rows:
        t0 = base[(x["rho_s_over_rho_l"], x["Ste"])]
        x["t_star"] = (x["t_fre"] - t0) / t0
    return rows


# Table 1 (Sec. 4): water on a wall at -10 C and hexadecane on a wall 3 K below its melting
# point, as the lattice groups they give: Stefan number, density, conductivity and heat
# capacity ratios of solid to liquid
COLD_WALL = {
    "water": {"Ste": 4220 * 10 / 333400, "rho": 917 / 999, "k": 2.16 / 0.581, "cp": 2100 / 4220},
    "hexadecane": {"Ste": 2310 * 3 / 230000, "rho": 833 / 774, "k": 0.15 / 0.15, "cp": 1800 / 2310},
}


def _apex_curvature(psi: np.ndarray, xc: float, half: int = 3) -> float:
    """Second difference of the top surface h(x) at the drop's centre column (h from the
    psi = 1/2 crossing of each column); a tip makes it large, a platform small."""
    ic = int(round(xc))
    hs = [drop_height(psi, {"xc": float(i)}) for i in range(ic - half, ic + half + 1, half)]
    return (hs[0] - 2 * hs[1] + hs[2]) / half ** 2


def contact_radius(psi: np.ndarray) -> float:
    """Half the psi >= 1/2 extent of the first row above the substrate."""
    return 0.5 * _span(psi[0, :])


def cold_wall(nx: int = 160, ny: int = 80, R0: float = 20.0, theta: float = 87.0,
              precision: str = "fp64", max_steps: int = 200000) -> list[dict]:
    """Sec. 4's sessile-drop freezing with Table 1's property ratios (no experimental overlay:
    those data are not available): each drop frozen completely as one batch; final material
    volume, height, contact radius and apex curvature relative to the start."""
    from .lbm import Batch
    names = list(COLD_WALL)
    cases = []
    for n in names:
        g = COLD_WALL[n]
        c = inputs.sessile_drop(nx, ny, R0, theta, 1.0, 1.0, 0.0, g["Ste"], seed=None,
                                rho_ratio_sl=g["rho"], k_ratio_sl=g["k"])
        c["cp_s"] = g["cp"] * c["cp_l"]
        cases.append(c)
    b = Batch(cases, precision=precision)
    start = []
    for k, c in enumerate(cases):
        psi = b.field(k, "psi")
        start.append((psi.clip(0, 1).sum(), drop_height(psi, c), contact_radius(psi),
                      _apex_curvature(psi, c["xc"])))
    b.run_until_frozen(max_steps)
    t_fre = [d["t_fre"] for d in b.diag()]
    steps = 0
    while steps < max_steps and not all(d["V_l"] < 1e-4 * d["V_l0"] for d in b.diag()):
        b.step(500)
        steps += 500
    out = []
    for k, (n, c) in enumerate(zip(names, cases)):
        psi = b.field(k, "psi")
        v0, h0, r0, a0 = start[k]
        out.append({"liquid": n, "Ste": COLD_WALL[n]["Ste"], "rho_s_over_rho_l": COLD_WALL[n]["rho"],
                    "t_fre": t_fre[k], "volume_ratio": float(psi.clip(0, 1).sum() / v0),
                    "closed_form_volume_ratio": 1.0 / COLD_WALL[n]["rho"],
                    "H_m_over_H_0": drop_height(psi, c) / h0, "R_tr_over_R_0": contact_radius(psi) / r0,
                    "apex_curvature": _apex_curvature(psi, c["xc"]), "apex_curvature_start": a0})
    return out
