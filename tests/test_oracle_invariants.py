"""Invariant pins of the oracle's coupled step (Algorithm 1): exact discrete conservation of
the phase-field populations, a uniform rest state that stays at rest, and mirror symmetry."""
import numpy as np
import pytest

from oracle import binding as ob
from oracle.binding import Oracle
from paper_2410_06657_amd import inputs


def _small_drop(rho_ratio=0.9, seed=None, nx=64, ny=32, R0=12.0, Ste=0.3, Ca_E=0.3):
    c = inputs.sessile_drop(nx, ny, R0, 90.0, 3.0, 1.0, Ca_E, Ste, seed=seed,
                            rho_ratio_sl=rho_ratio)
    c.update(poisson_tol=1e-10)
    return c


def test_phase_field_mass_is_conserved_without_volume_change(threads):
    """rho_s = rho_l gives mdot = 0: the populations f only collide (sum kept, Eqs. (18)-(19)
    with a zero source) and stream or bounce back, so sum f is constant."""
    o = Oracle(_small_drop(rho_ratio=1.0))
    s0 = o.pop("f").sum()
    o.step(200)
    assert o.diag()["V_s"] > 1.0  # the drop did freeze
    assert abs(o.pop("f").sum() - s0) <= 1e-12 * s0


def check_mass_budget(L=None, steps=60):
    """With freezing expansion the total of f changes every step by
    sum psi^n [mdot^n + (mdot^{n-1} - mdot^n)/(2 tau_f)] (collision of Eqs. (15), (19) with
    Eq. (20)); checked step by step."""
    c = _small_drop(rho_ratio=0.8)
    tau = c["M"] * 3 + 0.5
    o = Oracle(c, L=L)
    md_prev = np.zeros((c["ny"], c["nx"]))
    tot = o.pop("f").sum()
    for n in range(steps):
        psi, md = o.field("psi"), o.field("mdot")
        o.step(1)
        new = o.pop("f").sum()
        expect = tot + (psi * (md + (md_prev - md) / (2 * tau))).sum()
        assert abs(new - expect) <= 1e-12 * tot, n
        md_prev, tot = md, new
    assert np.abs(md_prev).max() > 0


def test_phase_field_mass_budget_with_volume_change(threads):
    check_mass_budget()


def test_uniform_rest_state_stays_at_rest():
    """All liquid at the melting point, equal electrode potentials, substrate at T_m: nothing
    drives the system, so every field stays where it started."""
    c = inputs.stefan_strip(8, 8, h0=1e6, Ste=0.0)
    c.update(phi_top=0.0, phi_bot=0.0, T_w=0.0, T_g=0.0)
    o = Oracle(c)
    before = {k: o.field(k) for k in ("psi", "ux", "uy", "p", "T", "H", "fs", "phi")}
    o.step(20)
    for k, v in before.items():
        np.testing.assert_allclose(o.field(k), v, atol=1e-14, err_msg=k)


def test_mirror_symmetry(threads):
    """A drop centred on a mirror line of the periodic lattice stays mirror symmetric:
    x -> nx - x maps the lattice onto itself and swaps the E/W and diagonal links."""
    c = _small_drop(seed=None)
    o = Oracle(c)
    o.step(100)
    nx = c["nx"]
    idx = (nx - np.arange(nx)) % nx
    for k in ("psi", "p", "T", "fs", "phi", "uy"):
        a = o.field(k)
        np.testing.assert_allclose(a, a[:, idx], atol=1e-12, err_msg=k)
    ux = o.field("ux")
    np.testing.assert_allclose(ux, -ux[:, idx], atol=1e-12)
    assert np.abs(ux).max() > 1e-6


def _centroid_x(psi):
    """x of the drop's centroid on the periodic axis (circular mean of the psi mass)."""
    nx = psi.shape[1]
    w = np.clip(psi, 0, 1).sum(axis=0)
    ang = 2 * np.pi * np.arange(nx) / nx
    a = np.arctan2((w * np.sin(ang)).sum(), (w * np.cos(ang)).sum())
    return (a % (2 * np.pi)) * nx / (2 * np.pi)


def check_drop_moves_with_the_flow(L=None, u0=0.005, steps=600):
    """Galilean pin of the phase-field forcing (Eqs. (19), (35)): a free drop in a uniform
    stream (every population at the equilibrium of u = u0, (psi u)^{n-1} = psi u0) is carried
    along at the stream's speed: measured 1.011 u0 t.  The box is tall enough that the no-slip
    walls' shear layers do not reach the drop within the run.  The stream is slow because the
    flow model's own high-order velocity errors at density ratio 10 speed the liquid up at
    faster streams (the flow inside the drop reaches 1.18 u0 after 500 steps at u0 = 0.02 and
    the drop 1.08 u0 t, against 1.005 u0 and 1.01 u0 t at u0 = 0.005); a sign error in the
    time derivative of psi u moves the drop at about 1.7 u0."""
    c = inputs.free_drop(128, 96, 12.0, R=1.0, S=1.0, Ca_E=0.0)
    o = Oracle(c, L=L)
    ny, nx = c["ny"], c["nx"]
    psi = o.field("psi")
    Cs, Cl, Cg = (c[f"rho_{k}"] * c[f"cp_{k}"] for k in "slg")
    Cref = 2 * Cs * Cl / (Cs + Cl)
    pc = psi.clip(0, 1)
    rho = pc * c["rho_l"] + (1 - pc) * c["rho_g"]
    Cv = pc * Cl + (1 - pc) * Cg
    H, T = o.field("H"), o.field("T")
    one = np.ones((ny, nx))
    o.set_field("ux", u0 * one)
    o.set_field("usx", u0 * one)
    o.set_field("psiu_x", psi * u0)
    f, h, g = (np.empty((9, ny, nx)) for _ in range(3))
    for j in range(ny):
        for i in range(nx):
            f[:, j, i] = ob.node_f(psi[j, i], u0, 0, 0, 0, 0, L=L)[0]
            h[:, j, i] = ob.node_h(0, rho[j, i], u0, 0, 0, 0, 0, 0, 0, L=L)[0]
            g[:, j, i] = ob.node_g(H[j, i], T[j, i], Cv[j, i], Cref, u0, 0, L=L)
    o.set_pop("f", f)
    o.set_pop("h", h)
    o.set_pop("g", g)
    x0 = _centroid_x(psi)
    o.step(steps)
    ratio = (_centroid_x(o.field("psi")) - x0) / (u0 * steps)
    print(f"drop speed / stream speed {ratio:.4f}")
    assert ratio == pytest.approx(1.0, abs=0.03)


def test_drop_moves_with_the_flow(threads):
    check_drop_moves_with_the_flow()
