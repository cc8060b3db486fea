"""Pins of the closed forms the validation runners compare against (no GPU): Neumann's root
against tabulated values and its small-Stefan limit, and the deformation formulas at values
computed by hand from their printed forms (Sec. 4)."""
import math

import pytest

from paper_2410_06657_amd import validation


def test_neumann_root():
    assert validation.neumann_lambda(0.1) == pytest.approx(0.2200162727, abs=1e-9)
    assert validation.neumann_lambda(0.2) == pytest.approx(0.3064239054, abs=1e-9)
    # small Ste: lambda -> sqrt(Ste / 2)
    assert validation.neumann_lambda(1e-4) / math.sqrt(0.5e-4) == pytest.approx(1, abs=1e-4)


def test_deformation_forms():
    # Feng: Ca f_F / (3 (1 + R)^2), f_F = R^2 + R + 1 - 3S
    assert validation.feng(3.0, 1.0, 0.1) == pytest.approx(0.1 * 10 / 48)
    assert validation.feng(0.5, 2.0, 0.3) == pytest.approx(-0.1888888889, rel=1e-9)
    # Taylor with B = 1: f_T = R^2 + 1 - 2S + 1.5 (R - S)
    assert validation.taylor(3.0, 1.0, 0.1) == pytest.approx(0.02475)
    assert validation.taylor(0.5, 2.0, 0.1) == pytest.approx(-0.045)
    # the prolate/oblate boundary of Feng's form
    assert validation.feng(5.0, 31.0 / 3.0, 0.2) == pytest.approx(0.0, abs=1e-15)


def test_measurement_helpers():
    import numpy as np
    # an ellipse psi field with semi-axes 12 (along y) and 10: D = (24 - 20) / 44
    ny = nx = 64
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c = {"xc": 32.0, "yc": 32.0}
    psi = 0.5 * (1 + np.tanh(2 * (1 - np.sqrt(((x - 32) / 10) ** 2 + ((y - 32) / 12) ** 2)) * 10 / 4))
    assert validation.deformation(psi, c) == pytest.approx(4 / 44, abs=2e-3)
    # an f_l profile linear around its 1/2 crossing at node coordinate 6.75, i.e. 7.25 from
    # the wall at -1/2
    fl = np.clip((np.arange(32) - 6.75) / 4.0 + 0.5, 0, 1)
    assert validation.front(fl) == pytest.approx(7.25, abs=1e-12)


def test_substrate_heat_flux_and_freezing_time_law():
    import numpy as np
    # the second-order one-sided difference is exact for a quadratic profile in y:
    # T = 1 + 0.3 j + 0.05 j^2 has dT/dy = 0.3 at j = 0
    ny, nx = 8, 6
    j = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    T = 1.0 + 0.3 * j + 0.05 * j ** 2
    case = {"k_l": 2.0, "k_g": 0.5, "k_s": 4.0}
    psi = np.zeros((ny, nx))
    psi[0, :3] = 1.0            # liquid over the first three columns, gas beyond
    fs = np.zeros((ny, nx))
    fs[0, 1] = 1.0              # one solid column
    q = validation.substrate_heat_flux(T, psi, fs, case)
    assert q == pytest.approx(0.3 * np.array([2.0, 4.0, 2.0, 0.5, 0.5, 0.5]), rel=1e-12)
    # rows that follow H_m/R_0 = C (Ste Fo)^(1/2) exactly: slope 1/2, no spread
    rows = [{"Ste": s, "Fo": fo, "H_m_over_R_0": 1.7 * math.sqrt(s * fo)}
            for s, fo in ((0.05, 4.0), (0.1, 1.5), (0.2, 3.0), (0.5, 0.4))]
    law = validation.ste_fo_law(rows)
    assert law["slope"] == pytest.approx(0.5, abs=1e-12)
    assert law["coefficient_spread"] == pytest.approx(1.0, abs=1e-12)
    assert law["coefficient_mean"] == pytest.approx(1.7, rel=1e-12)
