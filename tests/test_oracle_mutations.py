"""The pins have teeth: each case plants one plausible mistake in a copy of the oracle's
source (a flipped sign, a dropped term, a wrong weight or index), builds it, and shows that a
named pin of the real oracle fails on it.  Only the copy is changed; the oracle itself is
untouched.  Each case names the passage of the paper the planted line implements."""
import os

import pytest

from oracle import binding as ob
from oracle import build as obuild

import test_oracle_budgets as budgets
import test_oracle_ehd as ehd
import test_oracle_enthalpy as enthalpy
import test_oracle_invariants as invariants
import test_oracle_moments as moments
import test_oracle_physics as physics
import test_oracle_potential as potential
import test_oracle_wetting as wetting

SRC = os.path.join(os.path.dirname(obuild.__file__), "lbm_oracle.c")

# name: (line fragment, planted replacement, pin that must fail)
MUTATIONS = {
    "wetting ghost sign (wetting step of Algorithm 1)": (
        "gb = b + s->wet * b * (1 - b);", "gb = b - s->wet * b * (1 - b);",
        lambda L: wetting.check_contact_angle(90.0, 60.0, L)),
    "solid drag dropped from F + rho f (Eqs. (24), (26))": (
        "double Gx = s->Fx[n] + rho * fsx;", "double Gx = s->Fx[n];",
        lambda L: budgets.check_drag(1.0, L)),
    "half solid force dropped from u (Eq. (26))": (
        "ux[n] = ax + 0.5 * fs[n] * (0 - ax);", "ux[n] = ax;",
        lambda L: budgets.check_drag(0.5, L)),
    "S/2 dropped from the pressure (Eq. (27))": (
        "s0 + 0.5 * s->S[n] + s->tauh[n] * s->R0[n] + rho * s0u",
        "s0 + s->tauh[n] * s->R0[n] + rho * s0u",
        lambda L: budgets.check_volume_source(-0.02, L)),
    "tau R_0 dropped from the pressure (Eq. (27))": (
        "s0 + 0.5 * s->S[n] + s->tauh[n] * s->R0[n] + rho * s0u", "s0 + 0.5 * s->S[n] + rho * s0u",
        lambda L: budgets.check_volume_source(-0.02, L)),
    "forcing factor 1 - 1/(2 tau_f) dropped (Eq. (15))": (
        "(1 - 0.5 / tauf) * F[q]", "F[q]",
        lambda L: budgets.check_volume_source(-0.02, L)),
    "psi taken as sum f, the implicit source term dropped (Eq. (20))": (
        "psi[n] = sum / (1 - 0.5 * md[n]);", "psi[n] = sum;",
        lambda L: budgets.check_volume_source(-0.02, L)),
    "wrong weight in the enthalpy rest equilibrium (Eq. (29))": (
        "geq[0] = H - Cref * T + WQ[0] * (Cref * T", "geq[0] = H - Cref * T + WQ[1] * (Cref * T",
        lambda L: budgets.check_enthalpy_budget(L, steps=5)),
    "substrate temperature entering once, not twice (anti-bounce-back)": (
        "-src[OPP[q] * N + n] + 2 * WQ[q] * wallv", "-src[OPP[q] * N + n] + WQ[q] * wallv",
        lambda L: budgets.check_enthalpy_budget(L, steps=5)),
    "electrode anti-bounce-back sign (Sec. 3.4)": (
        "-lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_bot",
        "lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_bot",
        lambda L: potential.check_linear_fixed_point(L)),
    "top electrode anti-bounce-back sign (Sec. 3.4)": (
        "-lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_top",
        "lt[(size_t)LOPP[q] * N + n] + 2 * LW[q] * p->phi_top",
        lambda L: potential.check_alternating_sum(L)),
    "sign of the gradient-energy term of mu (Eq. (4))": (
        "- kap * lap;", "+ kap * lap;",
        lambda L: physics.check_laplace(L)),
    "sign of the dielectric force (Eq. (14))": (
        "s->Fy[n] += qv * Ey - 0.5 * E2 * gey;", "s->Fy[n] += qv * Ey + 0.5 * E2 * gey;",
        lambda L: ehd.check_feng(0.5, 2.0, L)),  # S = 2: grad(eps) is not zero
    "sign of the free charge (Eq. (14), q_v = div(eps E))": (
        "double qv = -(gex * gpx + gey * gpy + eps * lphi);",
        "double qv = (gex * gpx + gey * gpy + eps * lphi);",
        lambda L: ehd.check_feng(3.0, 1.0, L)),
    "rest weight of the flow equilibrium (Eq. (22))": (
        "heq[q] = p / CS2 * (WQ[q] - 1) + rho * s;", "heq[q] = p / CS2 * (WQ[q] + 1) + rho * s;",
        lambda L: moments.check_flow_moments(L=L)),
    "sign inside the second-order forcing term (Eq. (24))": (
        "double sec = (2 * cu * cF - 2 * CS2 * uF) / (2 * CS2 * CS2);",
        "double sec = (2 * cu * cF + 2 * CS2 * uF) / (2 * CS2 * CS2);",
        lambda L: moments.check_flow_moments(L=L)),
    "heat capacity of the frozen branch (Eq. (7))": (
        "double Csol = mix(Cs, Cl, Cg, pc, pc);", "double Csol = mix(Cs, Cl, Cg, pc, 0);",
        lambda L: enthalpy.check_round_trip(1.0, -0.3, L)),
    "sign of the previous level in d/dt(psi u) (Eq. (35))": (
        "double Ax = (ps * ux[n] - pux[n]) + CS2 * lam * nxv;",
        "double Ax = (ps * ux[n] + pux[n]) + CS2 * lam * nxv;",
        lambda L: invariants.check_drop_moves_with_the_flow(L)),
    "streaming pulls from the wrong side (Eq. (15))": (
        "v = src[q * N + (size_t)jj * nx + wrapx(i - CX[q], nx)];",
        "v = src[q * N + (size_t)jj * nx + wrapx(i + CX[q], nx)];",
        lambda L: wetting.check_contact_angle(90.0, 60.0, L)),
    "dynamic viscosity taken for the kinematic one in tau_h (Sec. 3.2)": (
        "double tauh = mu / (rho * CS2) + 0.5;", "double tauh = mu / CS2 + 0.5;",
        lambda L: physics.check_laplace(L)),
    "sign of the volume source (Eq. (2b))": (
        "md[n] = shrink * (fsn - fs[n]);", "md[n] = -shrink * (fsn - fs[n]);",
        lambda L: physics.check_final_height(0.9, L)),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_a_pin_catches_the_planted_mistake(name, tmp_path):
    frag, planted, check = MUTATIONS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(frag) == 1, "the line the case plants into is not in the oracle"
    src = tmp_path / "lbm_oracle.c"
    src.write_text(text.replace(frag, planted))
    L = ob.load(obuild.build(src=str(src), out=str(tmp_path / "libmutant.so")))
    ob.set_threads(min(8, os.cpu_count() or 1), L)
    with pytest.raises(AssertionError):
        check(L)
