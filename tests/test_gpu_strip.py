"""The 4 x 4096 Stefan strip (periodic across, freezing along the 4096 nodes) against the
one-phase Neumann solution (Sec. 4, three-phase Stefan problem without volume change): liquid
at the melting point on a substrate at T_w = -Ste, Ste = 0.1, alpha_s = 0.2; the front (the
f_l = 1/2 crossing) at s(t) = 2 lambda sqrt(alpha_s t) with lambda e^{lambda^2} erf(lambda) =
Ste / sqrt(pi).  Checked at s = 32 and 64 nodes (t = 26,444 and 105,774 steps) within 1% in
FP64, FP32 and FP32 with FP16 storage."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu


def front(fl):
    k = np.where(fl >= 0.5)[0][0]
    return (k - 1) + (0.5 - fl[k - 1]) / (fl[k] - fl[k - 1]) + 0.5


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16store"])
def test_strip_4x4096_follows_neumann(precision):
    from paper_2410_06657_amd.lbm import Solver
    ste, alpha = 0.1, 0.2
    lam = brentq(lambda x: x * math.exp(x * x) * math.erf(x) - ste / math.sqrt(math.pi), 1e-9, 3)
    assert lam == pytest.approx(0.2200162727, abs=1e-9)
    c = inputs.strip_4x4096(ny=4096, Ste=ste)
    assert (c["nx"], c["ny"]) == (4, 4096) and c["k_s"] / (c["rho_s"] * c["cp_s"]) == pytest.approx(alpha)
    g = Solver(c, precision)
    done = 0
    for s_target in (32.0, 64.0):
        t = int(round((s_target / (2 * lam)) ** 2 / alpha))
        g.step(t - done)
        done = t
        s = front(g.field("fl")[:, 0])
        exact = 2 * lam * math.sqrt(alpha * t)
        print(f"{precision}: t = {t}, front {s:.3f}, Neumann {exact:.3f}, rel {s / exact - 1:+.2e}", flush=True)
        assert s == pytest.approx(exact, rel=0.01)
