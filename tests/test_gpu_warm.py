"""Learned warm start: the committed network (trained on the GPU by the library's own kernels
on potentials the method produced; see paper_2410_06657_amd/warm.py) seeds the potential of
held-out drops, after which the plain sweeps run to the same stopping rule.  What the network
gains over the method without it: far fewer sweeps for the initial solve, with a final
potential as close to a tightly converged reference as the cold start's."""
import numpy as np
import pytest

from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu

CAP = 4000000


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("R,S,theta", [(3.0, 1.0, 90.0), (0.5, 2.0, 120.0)])
def test_warm_start_saves_sweeps_at_t0(R, S, theta):
    from paper_2410_06657_amd import warm
    from paper_2410_06657_amd.lbm import Solver
    nx, ny = 512, 256
    f = warm.factor_for(ny)
    net = warm.load((nx // f) * (ny // f))
    c = inputs.sessile_drop(nx, ny, 0.3125 * ny, theta, R, S, 0.1, 0.1, seed=77)
    c.update(poisson_max_sweeps=CAP)
    cold = Solver(c)
    kc = int(cold.sweep_log()[0])
    w = Solver(dict(c, skip_initial_solve=1))
    assert int(w.sweep_log()[0]) == 0
    w.warm_start(net, f)
    rc, kw, r = w.solve_potential(c["poisson_tol"], CAP)
    ref = Solver(c)
    ref.solve_potential(1e-12, CAP)
    pr = ref.field("phi")
    ec, ew = rel(cold.field("phi"), pr), rel(w.field("phi"), pr)
    print(f"R={R} S={S}: cold {kc} sweeps (error {ec:.2e}), warm {kw} sweeps (error {ew:.2e})")
    assert rc == 0 and kc < CAP
    assert kw <= 0.6 * kc
    assert ew <= 1.5 * ec


def test_warm_start_before_every_step():
    """The per-step hook: each step's solve starts from the network's seed instead of the
    previous potential and still runs to the stopping rule; the trajectory stays with the
    plain method's to the accuracy that rule gives."""
    from paper_2410_06657_amd import warm
    from paper_2410_06657_amd.lbm import Solver
    c = inputs.sessile_drop(256, 128, 40.0, 90.0, 3.0, 1.0, 0.2, 0.1, seed=78)
    f = warm.factor_for(128)
    net = warm.load((256 // f) * (128 // f))
    a, b = Solver(c), Solver(c)
    b.set_warm_start(net, f)
    a.step(10)
    b.step(10)
    ka, kb = a.sweep_log()[1:], b.sweep_log()[1:]
    print("sweeps per step: previous-step start", ka.tolist(), "network start", kb.tolist())
    assert a.diag()["noconv"] == 0 and b.diag()["noconv"] == 0
    assert rel(b.field("psi"), a.field("psi")) <= 1e-6
    assert rel(b.field("phi"), a.field("phi")) <= 1e-3
    b.set_warm_start(None)
    b.step(2)
    assert b.sweep_log()[-1] < kb.min()


def test_warm_start_fp32():
    """The FP32 form takes the seed as base/remainder link pairs and gains the same way."""
    from paper_2410_06657_amd import warm
    from paper_2410_06657_amd.lbm import Solver
    nx, ny = 512, 256
    f = warm.factor_for(ny)
    net = warm.load((nx // f) * (ny // f))
    c = inputs.sessile_drop(nx, ny, 0.3125 * ny, 90.0, 3.0, 1.0, 0.1, 0.1, seed=79)
    c.update(poisson_max_sweeps=CAP)
    cold = Solver(c, "fp32")
    kc = int(cold.sweep_log()[0])
    w = Solver(dict(c, skip_initial_solve=1), "fp32")
    w.warm_start(net, f)
    rc, kw, _ = w.solve_potential(c["poisson_tol"], CAP)
    e = rel(w.field("phi"), cold.field("phi"))
    print(f"fp32: cold {kc} sweeps, warm {kw} sweeps, phi difference {e:.2e}")
    assert rc == 0 and kw <= 0.6 * kc and e <= 1e-3
