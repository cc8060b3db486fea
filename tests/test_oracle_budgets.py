"""Exact discrete identities of the oracle's flow and enthalpy updates, derived by hand from
the printed scheme on states where the coupled step reduces to a few terms.

* Enthalpy (Sec. 3.3, Eqs. (28)-(30)): with rho_s = rho_l there is no volume source, so
  Q = C T mdot = 0; the collision keeps sum g (the equilibrium's zeroth moment is H) and
  streaming keeps it except at the substrate, where the anti-bounce-back of Eq. (28)'s wall
  rule replaces the three links leaving the domain by -g* + 2 w_i C_ref T_w.  Hence
  sum g^{n+1} - sum g^n = -2 sum_{substrate row} (g*_S + g*_SW + g*_SE) + nx C_ref T_w / 3,
  with g* the post-collision populations of the step and the adiabatic top contributing
  nothing.
* Solid drag (Sec. 3.2, Eqs. (24)-(26) with u_s = 0): in a uniform region of solid fraction
  f_s with no other force, one step multiplies the momentum moment by exactly (1 - f_s):
  u*^{n+1} = (1 - f_s) u*^n, whatever tau_h.  (Collision: rho u* - omega (rho u* - rho u)
  + (1 - omega/2) rho f, with u = (1 - f_s/2) u* and f = -f_s u*.)  A fully solid region
  stops in one step.
* Volume source (Eqs. (19)-(20) with div u = mdot; Eqs. (24), (27)): a uniform liquid at rest
  with a prescribed source mdot gets, after one step,
  psi^{n+1} = (1 + (1 - 1/(2 tau_f)) mdot) / (1 - mdot/2)   (f: F_i = w_i psi mdot), and
  p^{n+1} = c_s^2 S [(1 - 1/(2 tau_h)) + (1/2 + tau_h w_0) / (1 - w_0)], S = rho mdot
  (h: R_i = w_i S; Eq. (27) adds S/2 and tau_h R_0 with R_0 = w_0 S to the sum of the
  moving links).  Each of Eq. (27)'s S/2 and tau R_0 terms moves p^{n+1} by a quarter or more.
"""
import numpy as np
import pytest

from oracle import binding as ob
from oracle.binding import Oracle
from paper_2410_06657_amd import inputs

CS2 = 1.0 / 3.0
W0 = 4.0 / 9.0


def check_enthalpy_budget(L=None, steps=40):
    """A freezing drop in the field with rho_s = rho_l: the step's change of sum g is the
    substrate's anti-bounce-back flux and nothing else, and the collision alone keeps sum g."""
    c = inputs.sessile_drop(64, 32, 10.0, 75.0, 3.0, 1.0, 0.2, 0.3, seed=3, rho_ratio_sl=1.0)
    o = Oracle(c, L=L)
    Cs, Cl = c["rho_s"] * c["cp_s"], c["rho_l"] * c["cp_l"]
    Cref = 2 * Cs * Cl / (Cs + Cl)
    nx = c["nx"]
    o.step(5)
    for n in range(steps):
        g0 = o.pop("g").sum()
        o.step(1)
        gp = o.pop("g_post")
        g1 = o.pop("g").sum()
        assert abs(gp.sum() - g0) <= 1e-13 * abs(g0), n
        out = gp[[4, 7, 8], 0, :].sum()
        expect = g0 - 2 * out + nx * Cref * c["T_w"] / 3
        assert abs(g1 - expect) <= 1e-13 * abs(g0), (n, g1 - expect)
    d = o.diag()
    assert d["V_s"] > 0.5 and np.abs(o.field("mdot")).max() == 0.0


def test_enthalpy_budget_at_the_walls(threads):
    check_enthalpy_budget()


def uniform_case(nx=8, ny=8, **kw):
    """A column entirely of condensed phase (psi = 1), equal densities everywhere, no field,
    everything at the melting point."""
    c = inputs.stefan_strip(nx, ny, h0=1e6, Ste=0.0)
    c.update(rho_s=1.0, rho_g=1.0, T_g=0.0, T_w=0.0, phi_top=0.0, phi_bot=0.0)
    c.update(kw)
    return c


def check_drag(fs, L=None):
    c = uniform_case(ny=16)
    o = Oracle(c, L=L)
    ny, nx = c["ny"], c["nx"]
    Lvol = c["rho_s"] * c["latent"]
    u0 = 0.02
    us = u0
    u = (1 - fs / 2) * u0
    one = np.ones((ny, nx))
    o.set_field("fs", fs * one)
    o.set_field("fl", (1 - fs) * one)
    o.set_field("H", (1 - fs) * Lvol * one)
    o.set_field("T", 0 * one)
    o.set_field("usx", us * one)
    o.set_field("ux", u * one)
    o.set_field("psiu_x", u * one)  # d/dt(psi u) = 0
    feq, _ = ob.node_f(1.0, u, 0.0, 0.0, 0.0, 0.0, L=L)
    heq, _ = ob.node_h(0.0, 1.0, us, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, L=L)
    geq = np.zeros(9)
    geq[0] = (1 - fs) * Lvol
    o.set_pop("f", feq[:, None, None] * one)
    o.set_pop("h", heq[:, None, None] * one)
    o.set_pop("g", geq[:, None, None] * one)
    for k in (1, 2):
        o.step(1)
        # rows the walls have not reached yet: a step carries their influence two rows in
        # (one through the pressure stencil of F~, one by streaming)
        inner = slice(2 * k, ny - 2 * k)
        got = o.field("usx")[inner]
        np.testing.assert_allclose(got, (1 - fs) ** k * u0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(o.field("ux")[inner], (1 - fs / 2) * (1 - fs) ** k * u0, atol=1e-15)
        np.testing.assert_allclose(o.field("fs")[inner], fs, atol=1e-15)


@pytest.mark.parametrize("fs", [1.0, 0.5, 0.25])
def test_solid_drag_removes_momentum_at_rate_fs(fs):
    check_drag(fs)


def check_volume_source(mdot, L=None):
    c = uniform_case()
    o = Oracle(c, L=L)
    ny, nx = c["ny"], c["nx"]
    one = np.ones((ny, nx))
    o.set_field("mdot", mdot * one)
    o.step(1)
    tau_f = c["M"] / CS2 + 0.5
    tau_h = c["mu_l"] / (1.0 * CS2) + 0.5
    psi1 = (1 + (1 - 0.5 / tau_f) * mdot) / (1 - 0.5 * mdot)
    S = 1.0 * mdot
    p1 = CS2 * S * ((1 - 0.5 / tau_h) + (0.5 + tau_h * W0) / (1 - W0))
    np.testing.assert_allclose(o.field("psi"), psi1, rtol=1e-14)
    np.testing.assert_allclose(o.field("p"), p1, rtol=1e-12)
    np.testing.assert_allclose(o.field("uy"), 0.0, atol=1e-18)
    # each of the printed S/2 and tau R_0 terms carries a quarter or more of p^{n+1}
    assert abs(CS2 * S * 0.5 / (1 - W0)) > 0.25 * abs(p1)
    assert abs(CS2 * S * tau_h * W0 / (1 - W0)) > 0.25 * abs(p1)


@pytest.mark.parametrize("mdot", [-0.02, 0.01])
def test_uniform_volume_source_one_step(mdot):
    check_volume_source(mdot)
