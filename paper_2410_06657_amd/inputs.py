"""Seeded synthetic cases for the electrofreezing lattice Boltzmann path.

This module only describes problems: it maps the paper's dimensionless groups to
lattice-unit parameters and draws the seeded jitter of the droplet centre.  It holds none
of the method's arithmetic, and both the GPU library's binding and the CPU oracle's
binding consume the plain dicts it returns.

The paper fixes no lattice values (its Secs. 4-5 give only dimensionless groups), so the
defaults below are choices, each stated with its reason:

* W = 4, M = 0.1 (tau_f = 0.8), gamma = 0.01;
* rho_l = 1, rho_g = 0.1 (liquid/gas density ratio 10), rho_s/rho_l = 0.9 (Sec. 5,
  Figs. 7, 9-13) unless a case says otherwise;
* mu = 0.05 in every phase (viscosity ratio B = 1, as in the R-S diagram of Sec. 5);
* c_p = 1 in liquid and solid, c_p,gas = rho_l/rho_g, so that the volumetric heat
  capacity rho*c_p of the gas equals the liquid's.  The total-enthalpy scheme with a
  constant C_ref is unstable when C_ref is several times the local rho*c_p (the rest
  population of its equilibrium turns strongly negative); the paper gives no c_p for the
  gas, only alpha_l/alpha_g = 0.2, which is kept;
* latent heat L = 1, so Ste = c_p (T_m - T_w)/L gives T_w = -Ste (T_m = 0 datum);
* droplets start slightly above their melting point, T_g = 0.01 (the paper gives no T_g).
  With T_g = T_m exactly every node starts on the liquidus branch point of Eq. (7), where in
  the interface tails the mushy fraction H / (psi rho_s L) is a ratio of two tiny numbers:
  rounding noise in H is then amplified by 1/(psi rho_s L) and two FP64 runs that differ by
  1e-15 drift apart to ~1e-10 within 200 steps; with the superheat they stay within 1e-12
  over 1000 steps.  Stefan strips keep T_g = T_m (the one-phase Neumann problem);
* k_l = 0.1 (alpha_l = 0.1), k_s = 2 k_l (ice/liquid conductivity ratio 2),
  k_g = 5 alpha_l * rho_g c_p,g (alpha_l/alpha_g = 0.2, Sec. 5);
* sigma_gas = 1/6 (tau_l = 1 in the gas), sigma_drop = R sigma_gas, eps_drop = S eps_gas,
  solid = liquid for both (Table 1 gives no solid values);
* phi_top = 1, phi_bot = 0, E_0 = 1/ny, eps_gas = Ca_E gamma / (E_0^2 R0) from
  Ca_E = eps_e E_0^2 R / gamma (Sec. 4, deformation test);
* potential tolerance 1e-8 on the relative sweep-to-sweep change.
"""
from __future__ import annotations

import math

MASK64 = (1 << 64) - 1

# reading switch bits (same meaning on both sides; each side defines its own constant)
R_GRAD_S = 1


def splitmix64(state: int) -> tuple[int, int]:
    """One step of SplitMix64 (Steele, Lea, Flood 2014).  Returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def uniform(seed: int, k: int = 0) -> float:
    """k-th uniform [0, 1) double of the SplitMix64 stream seeded with `seed`."""
    s = seed & MASK64
    out = 0
    for _ in range(k + 1):
        s, out = splitmix64(s)
    return (out >> 11) * (1.0 / (1 << 53))


def base_params(nx: int, ny: int) -> dict:
    """Default lattice values; every case starts from these."""
    rho_l, rho_g = 1.0, 0.1
    alpha_l = 0.1
    cp_g = rho_l / rho_g
    return dict(
        nx=int(nx), ny=int(ny),
        W=4.0, M=0.1, gamma=0.01,
        rho_l=rho_l, rho_g=rho_g, rho_s=0.9,
        mu_l=0.05, mu_g=0.05, mu_s=0.05,
        cp_l=1.0, cp_g=cp_g, cp_s=1.0,
        k_l=alpha_l * rho_l * 1.0, k_s=2 * alpha_l * rho_l * 1.0,
        k_g=(alpha_l / 0.2) * rho_g * cp_g,
        latent=1.0,
        T_w=-0.1, T_g=0.0,
        eps_l=0.0, eps_g=0.0, eps_s=0.0,
        sig_l=1.0 / 6, sig_g=1.0 / 6, sig_s=1.0 / 6,
        phi_top=1.0, phi_bot=0.0,
        theta_deg=90.0,
        shape=0, R0=0.0, xc=0.0, yc=0.0, h0=0.0,
        poisson_tol=1e-8, poisson_max_sweeps=200000,
        readings=R_GRAD_S,
    )


def set_electric(case: dict, R: float, S: float, Ca_E: float, R0: float) -> dict:
    """Conductivity ratio R, permittivity ratio S and electric capillary number Ca_E."""
    E0 = (case["phi_top"] - case["phi_bot"]) / case["ny"]
    eps_e = Ca_E * case["gamma"] / (E0 * E0 * R0) if Ca_E > 0 else 0.0
    sig_e = 1.0 / 6
    case.update(eps_g=eps_e, eps_l=S * eps_e, eps_s=S * eps_e,
                sig_g=sig_e, sig_l=R * sig_e, sig_s=R * sig_e)
    return case


def sessile_drop(nx: int, ny: int, R0: float, theta_deg: float, R: float, S: float,
                 Ca_E: float, Ste: float, seed: int | None = None,
                 rho_ratio_sl: float = 0.9, k_ratio_sl: float = 2.0,
                 T_g: float = 0.01) -> dict:
    """A spherical cap of curvature radius R0 resting on the cooled substrate at angle theta.

    The centre sits at x = nx/2 + delta with delta ~ U[-1/2, 1/2) drawn from SplitMix64(seed)
    (no jitter when seed is None) and at y = -1/2 - R0 cos(theta), the wall being y = -1/2.
    """
    c = base_params(nx, ny)
    delta = 0.0 if seed is None else uniform(seed) - 0.5
    c.update(shape=0, R0=float(R0), xc=nx / 2 + delta,
             yc=-0.5 - R0 * math.cos(math.radians(theta_deg)), theta_deg=float(theta_deg),
             T_w=-float(Ste), T_g=float(T_g), rho_s=rho_ratio_sl * c["rho_l"],
             k_s=k_ratio_sl * c["k_l"])
    set_electric(c, R, S, Ca_E, R0)
    c["seed"] = seed
    return c


def free_drop(nx: int, ny: int, R0: float, R: float, S: float, Ca_E: float) -> dict:
    """A free (suspended) drop in the middle of the box, no freezing (T_w = T_g > T_m)."""
    c = base_params(nx, ny)
    c.update(shape=0, R0=float(R0), xc=nx / 2, yc=(ny - 1) / 2, theta_deg=90.0,
             T_w=0.5, T_g=0.5, rho_s=c["rho_l"])
    set_electric(c, R, S, Ca_E, R0)
    return c


def stefan_strip(nx: int, ny: int, h0: float, Ste: float, rho_ratio_sl: float = 1.0,
                 alpha_s: float | None = None) -> dict:
    """Liquid layer of thickness h0 on the cold substrate, gas above, no electric field."""
    c = base_params(nx, ny)
    c.update(shape=1, h0=float(h0), T_w=-float(Ste), rho_s=rho_ratio_sl * c["rho_l"],
             theta_deg=90.0)
    if alpha_s is not None:
        c["k_s"] = alpha_s * c["rho_s"] * c["cp_s"]
    set_electric(c, 1.0, 1.0, 0.0, 1.0)
    return c


# ---- the five workloads -------------------------------------------------------------------

def drop_128x64(seed: int = 0) -> dict:
    """128x64 FP64 sessile drop: R0 = 24, theta = 90, W = 4, Ste = 0.1, R = 3, S = 1 (prolate),
    Ca_E = 0.1, potential to 1e-8 every step, centre jitter from the seed."""
    return sessile_drop(128, 64, 24.0, 90.0, 3.0, 1.0, 0.1, 0.1, seed=seed)


DROP_1024_THETAS = (60.0, 90.0, 120.0)
DROP_1024_PAIRS = {"prolate": (3.0, 1.0), "oblate": (0.5, 2.0)}
DROP_1024_CAE = (0.0, 0.1, 0.3)


def drop_1024x512(theta_deg: float = 90.0, kind: str = "prolate", Ca_E: float = 0.1) -> dict:
    """1024x512, R0 = 160; prolate (R=3, S=1) or oblate (R=0.5, S=2); Ca_E in {0, 0.1, 0.3};
    liquid/gas density 10, ice/liquid conductivity 2, Ste = 0.1."""
    R, S = DROP_1024_PAIRS[kind]
    return sessile_drop(1024, 512, 160.0, theta_deg, R, S, Ca_E, 0.1, seed=0)


def drop_4096x2048() -> dict:
    """4096x2048, R0 = 640, theta = 90, R = 3, S = 1, Ca_E = 0.1, Ste = 0.1."""
    return sessile_drop(4096, 2048, 640.0, 90.0, 3.0, 1.0, 0.1, 0.1, seed=0)


def strip_4x4096(ny: int = 4096, h0: float | None = None, Ste: float = 0.1,
               rho_ratio_sl: float = 1.0) -> dict:
    """The 4 x 4096 Stefan strip (periodic in x, freezing along y)."""
    return stefan_strip(4, ny, h0 if h0 is not None else ny - 8, Ste, rho_ratio_sl)


def drop_batch(seed: int = 4, ncases: int = 96) -> list:
    """The batched sweep: ncases sessile drops with N_y ~ U{128, 144, ..., 768}, N_x = 2 N_y,
    R0 = 0.3125 N_y, Ca_E ~ U[0, 0.4], theta ~ U[45, 135] deg, R ~ logU[0.3, 5],
    S ~ logU[0.5, 3], Ste = 0.1, FP32.  Case c uses uniforms 5c .. 5c+4 of SplitMix64(seed)
    and seeds its centre jitter with 1000 seed + c."""
    cases = []
    s = seed & MASK64
    draws = []
    for _ in range(5 * ncases):
        s, out = splitmix64(s)
        draws.append((out >> 11) * (1.0 / (1 << 53)))
    for c in range(ncases):
        u = draws[5 * c:5 * c + 5]
        ny = 128 + 16 * min(int(u[0] * 41), 40)
        nx = 2 * ny
        Ca = 0.4 * u[1]
        theta = 45.0 + 90.0 * u[2]
        R = math.exp(math.log(0.3) + u[3] * (math.log(5.0) - math.log(0.3)))
        S = math.exp(math.log(0.5) + u[4] * (math.log(3.0) - math.log(0.5)))
        case = sessile_drop(nx, ny, 0.3125 * ny, theta, R, S, Ca, 0.1, seed=1000 * seed + c)
        cases.append(case)
    return cases


def scaled(case: dict, nx: int, ny: int) -> dict:
    """The same droplet problem on another grid: lengths scale with ny."""
    f = ny / case["ny"]
    c = dict(case)
    c.update(nx=int(nx), ny=int(ny), R0=case["R0"] * f,
             xc=nx / 2 + (case["xc"] - case["nx"] / 2),
             yc=-0.5 - (-0.5 - case["yc"]) * f)
    # E_0 = 1/ny changes with the grid; keep Ca_E by rescaling the permittivities
    Ca_scale = (ny / case["ny"]) ** 2 / f
    for k in ("eps_l", "eps_g", "eps_s"):
        c[k] = case[k] * Ca_scale
    return c
