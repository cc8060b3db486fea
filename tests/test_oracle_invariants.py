"""Invariant pins of the oracle's coupled step (Algorithm 1): exact discrete conservation of
the phase-field populations, a uniform rest state that stays at rest, and mirror symmetry."""
import numpy as np
import pytest

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


def test_phase_field_mass_budget_with_volume_change(threads):
    """With freezing expansion the total of f changes every step by
    sum psi^n [mdot^n + (mdot^{n-1} - mdot^n)/(2 tau_f)] (collision of Eqs. (15), (19) with
    Eq. (20)); checked step by step."""
    c = _small_drop(rho_ratio=0.8)
    tau = c["M"] * 3 + 0.5
    o = Oracle(c)
    md_prev = np.zeros((c["ny"], c["nx"]))
    tot = o.pop("f").sum()
    for n in range(60):
        psi, md = o.field("psi"), o.field("mdot")
        o.step(1)
        new = o.pop("f").sum()
        expect = tot + (psi * (md + (md_prev - md) / (2 * tau))).sum()
        assert abs(new - expect) <= 1e-12 * tot, n
        md_prev, tot = md, new
    assert np.abs(md_prev).max() > 0


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
