"""Pin of the oracle's wetting condition (Algorithm 1, wetting step; the cubic wall energy
consistent with Eq. (5)): with no field, no freezing and equal densities, a drop resting on the
substrate relaxes to the prescribed equilibrium contact angle.  The angle is measured on the
psi = 1/2 contour: a circle fitted to the contour points at least 4 nodes above the wall
(y >= 3.5), whose centre height yc and radius R give cos(theta) = (y_w - yc) / R with the wall
at y_w = -1/2.  Each case starts from a cap at another angle, so the drop has to move to the
prescribed one: a sign error in the ghost rule would send it to 180 - theta, a missing factor
to a different angle."""
import math

import numpy as np
import pytest

from oracle.binding import Oracle
from paper_2410_06657_amd import inputs


def contour_points(psi):
    """Points where psi crosses 1/2 between horizontal or vertical neighbours (linear
    interpolation; x periodic)."""
    ny, nx = psi.shape
    a, b = psi, np.roll(psi, -1, axis=1)
    j, i = np.nonzero((a - 0.5) * (b - 0.5) < 0)
    xs = i + (a[j, i] - 0.5) / (a[j, i] - b[j, i])
    pts = [np.c_[xs, j.astype(float)]]
    a, b = psi[:-1], psi[1:]
    j, i = np.nonzero((a - 0.5) * (b - 0.5) < 0)
    ys = j + (a[j, i] - 0.5) / (a[j, i] - b[j, i])
    pts.append(np.c_[i.astype(float), ys])
    return np.vstack(pts)


def cap_angle(psi, ymin=3.5):
    """Contact angle (degrees) of the drop from a least-squares circle through its contour."""
    p = contour_points(psi)
    p = p[p[:, 1] >= ymin]
    x, y = p[:, 0], p[:, 1]
    A = np.c_[2 * x, 2 * y, np.ones_like(x)]
    cx, cy, c0 = np.linalg.lstsq(A, x * x + y * y, rcond=None)[0]
    R = math.sqrt(c0 + cx * cx + cy * cy)
    return math.degrees(math.acos(np.clip((-0.5 - cy) / R, -1.0, 1.0)))


def test_circle_fit_recovers_a_known_cap():
    """The measurement itself: an initial tanh cap at 60 degrees reads back as 60."""
    c = inputs.sessile_drop(96, 40, 14.0, 60.0, 1.0, 1.0, 0.0, 0.0, seed=None, rho_ratio_sl=1.0, T_g=0.5)
    o = Oracle(dict(c, T_w=0.5))
    assert cap_angle(o.field("psi")) == pytest.approx(60.0, abs=0.2)


def realised_angle(start, theta, L=None, steps=6000):
    """Contact angle of a drop started as a cap at `start` degrees on a substrate that
    prescribes `theta`, after `steps` steps without cooling or field."""
    R0 = 16.0 if start == 90.0 else 14.0
    c = inputs.sessile_drop(96, 40, R0, start, 1.0, 1.0, 0.0, 0.0, seed=None, rho_ratio_sl=1.0, T_g=0.5)
    c.update(theta_deg=theta, T_w=0.5)  # no cooling, no field: only capillarity and wetting
    o = Oracle(c, L=L)
    o.step(steps)
    assert o.diag()["V_s"] == 0.0
    return cap_angle(o.field("psi"))


def check_contact_angle(start, theta, L=None):
    got = realised_angle(start, theta, L)
    print(f"start {start}, prescribed {theta}, realised {got:.2f}")
    assert got == pytest.approx(theta, abs=2.0)


@pytest.mark.parametrize("start,theta", [(90.0, 60.0), (90.0, 120.0), (60.0, 90.0)])
def test_drop_relaxes_to_the_prescribed_contact_angle(threads, start, theta):
    check_contact_angle(start, theta)
