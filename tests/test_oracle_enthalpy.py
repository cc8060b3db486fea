"""Pins of the oracle's enthalpy inversion, Eq. (7), on the volumetric enthalpy: every branch
returns the (T, f_l) the enthalpy was built from, and the map is continuous at the solidus
and liquidus enthalpies."""
import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs


def _caps(c, psi, fs):
    pc = min(max(psi, 0), 1)
    mix = lambda s, l, g: fs * s + (1 - fs) * pc * l + (1 - fs) * (1 - pc) * g
    return mix(c["rho_s"] * c["cp_s"], c["rho_l"] * c["cp_l"], c["rho_g"] * c["cp_g"])


def check_round_trip(psi, T, L=None):
    c = inputs.base_params(8, 8)
    Leff = psi * c["rho_s"] * c["latent"]
    if T < 0:
        H = _caps(c, psi, psi) * T  # all the node's liquid frozen
        Tr, fl = ob.invert_enthalpy(c, H, psi, L=L)
        assert fl == 0 and Tr == pytest.approx(T, rel=1e-14)
    else:
        H = _caps(c, psi, 0) * T + Leff
        Tr, fl = ob.invert_enthalpy(c, H, psi, L=L)
        assert fl == 1 and Tr == pytest.approx(T, rel=1e-14)


@pytest.mark.parametrize("psi", [1.0, 0.7, 0.3])
@pytest.mark.parametrize("T", [-0.3, -0.01, 0.02, 0.4])
def test_round_trip(psi, T):
    check_round_trip(psi, T)


@pytest.mark.parametrize("frac", [0.0, 0.25, 0.5, 1.0])
def test_mushy_branch(frac):
    c = inputs.base_params(8, 8)
    Leff = 0.8 * c["rho_s"] * c["latent"]
    T, fl = ob.invert_enthalpy(c, frac * Leff, 0.8)
    assert T == 0 and fl == pytest.approx(frac, abs=1e-15)


def test_continuity_and_gas():
    c = inputs.base_params(8, 8)
    Leff = c["rho_s"] * c["latent"]
    for H, side in [(0.0, "solidus"), (Leff, "liquidus")]:
        a = ob.invert_enthalpy(c, H - 1e-12, 1.0)
        b = ob.invert_enthalpy(c, H + 1e-12, 1.0)
        assert abs(a[0] - b[0]) < 1e-10 and abs(a[1] - b[1]) < 1e-10, side
    # pure gas carries no latent heat: any H >= 0 is "liquid" (no solid forms in the gas)
    T, fl = ob.invert_enthalpy(c, 0.05, 0.0)
    assert fl == 1 and T == pytest.approx(0.05 / (c["rho_g"] * c["cp_g"]))
    T, fl = ob.invert_enthalpy(c, -0.05, 0.0)
    assert fl == 0 and T == pytest.approx(-0.05 / (c["rho_g"] * c["cp_g"]))
