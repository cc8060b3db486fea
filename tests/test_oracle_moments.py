"""Pins of the oracle's node-level equilibria and forcing terms: the moment identities that
each equilibrium of Sec. 3 is built to satisfy (exact, checked on random inputs)."""
import numpy as np
import pytest

from oracle import binding as ob

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
CS2 = 1.0 / 3.0
RNG = np.random.default_rng(1234)


def _moments(a):
    return (a.sum(), (CX * a).sum(), (CY * a).sum(),
            (CX * CX * a).sum(), (CX * CY * a).sum(), (CY * CY * a).sum())


def test_lattice_directions_follow_eq17():
    """Eq. (17): axis links at angles (i-1) pi/2, diagonals at (2i-9) pi/4 with length sqrt 2."""
    for i in range(1, 5):
        ang = (i - 1) * np.pi / 2
        assert (CX[i], CY[i]) == (round(np.cos(ang)), round(np.sin(ang)))
    for i in range(5, 9):
        ang = (2 * i - 9) * np.pi / 4
        assert (CX[i], CY[i]) == (round(np.sqrt(2) * np.cos(ang)), round(np.sqrt(2) * np.sin(ang)))


@pytest.mark.parametrize("trial", range(20))
def test_phase_field_moments(trial):
    """Eqs. (18)-(19): sum f_eq = psi, sum c f_eq = psi u, sum c c f_eq = c_s^2 psi I;
    sum F = psi mdot, sum c F = d(psi u)/dt + c_s^2 lambda n."""
    psi, ux, uy, Ax, Ay, md = RNG.normal(size=6) * [1, 0.1, 0.1, 0.01, 0.01, 0.01]
    feq, F = ob.node_f(psi, ux, uy, Ax, Ay, md)
    m = _moments(feq)
    np.testing.assert_allclose(m, [psi, psi * ux, psi * uy, CS2 * psi, 0, CS2 * psi], atol=1e-15)
    m = _moments(F)
    np.testing.assert_allclose(m[:3], [psi * md, Ax, Ay], atol=1e-15)


def check_flow_moments(rng=RNG, L=None):
    """Eqs. (22)-(24): sum h_eq = 0, sum c h_eq = rho u, sum c c h_eq = p I + rho u u;
    sum R = S, sum c R = F + rho f, sum c c R = c_s^2 S I + u F~ + F~ u."""
    p, rho, ux, uy, S, Ftx, Fty, Gx, Gy = rng.normal(size=9) * 0.05
    rho = 0.1 + abs(rho) * 10
    heq, R = ob.node_h(p, rho, ux, uy, S, Ftx, Fty, Gx, Gy, L=L)
    m = _moments(heq)
    exp = [0, rho * ux, rho * uy, p + rho * ux * ux, rho * ux * uy, p + rho * uy * uy]
    np.testing.assert_allclose(m, exp, atol=1e-15)
    m = _moments(R)
    exp = [S, Gx, Gy, CS2 * S + 2 * ux * Ftx, ux * Fty + Ftx * uy, CS2 * S + 2 * uy * Fty]
    np.testing.assert_allclose(m, exp, atol=1e-15)


@pytest.mark.parametrize("trial", range(20))
def test_flow_moments(trial):
    check_flow_moments()


@pytest.mark.parametrize("trial", range(20))
def test_enthalpy_moments(trial):
    """Eq. (29): sum g_eq = H, sum c g_eq = C T u, sum c c g_eq = C_ref T c_s^2 I + C T u u."""
    H, T, ux, uy = RNG.normal(size=4) * [1, 0.1, 0.05, 0.05]
    Cv, Cref = 0.5 + RNG.random(2)
    geq = ob.node_g(H, T, Cv, Cref, ux, uy)
    m = _moments(geq)
    exp = [H, Cv * T * ux, Cv * T * uy, Cref * T * CS2 + Cv * T * ux * ux,
           Cv * T * ux * uy, Cref * T * CS2 + Cv * T * uy * uy]
    np.testing.assert_allclose(m, exp, atol=1e-14)


@pytest.mark.parametrize("phi", [0.0, 1.0, -0.37, 12.5])
def test_potential_equilibrium(phi):
    """Eqs. (32)-(34): the D2Q5 equilibrium sums to zero, its moving part gives phi back and
    its second moment is c_s^2 phi I with c_s^2 = 1/3."""
    leq = ob.node_l(phi)
    lx = np.array([0, 1, 0, -1, 0]); ly = np.array([0, 0, 1, 0, -1])
    assert abs(leq.sum()) <= 1e-15 * max(1, abs(phi))
    assert leq[1:].sum() / (1 - 1 / 3) == pytest.approx(phi, abs=1e-14)
    assert (lx * lx * leq).sum() == pytest.approx(phi / 3, abs=1e-14)
    assert (lx * leq).sum() == 0 and (ly * leq).sum() == 0
