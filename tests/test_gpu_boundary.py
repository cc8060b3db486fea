"""The C ABI's reporting and ownership rules, through the library itself:

* lbm_diag's operator residual of the potential equation (Sec. 2, in Eq. (36)'s discrete form)
  equals the oracle's, for the stepped state and after a tighter solve;
* a capped initial solve: lbm_init returns LBM_ENOCONV with a valid handle and
  lbm_diag.init_converged = 0;
* lbm_autotune runs in the caller's workspace (LBM_ESPACE if it is too small);
* lbm_get_field_device writes the same FP64 values as lbm_get_field, on the device;
* lbm_restore rejects an image with out-of-range buffer indices or from other parameters."""
import ctypes as C
import math
import os

import numpy as np
import pytest

from oracle import binding as ob
from paper_2410_06657_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads():
    ob.set_threads(min(16, os.cpu_count() or 1))
    yield
    ob.set_threads(1)


def small_drop(seed=0):
    return inputs.scaled(inputs.drop_128x64(seed), 96, 48)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_operator_residual_matches_oracle(precision, tol):
    from paper_2410_06657_amd.lbm import Solver
    c = small_drop(4)
    g, o = Solver(c, precision), ob.Oracle(c)
    g.step(6)
    o.step(6)
    for stage in ("stepped", "tight"):
        dg, do = g.diag(), o.diag()
        print(stage, precision, dg["op_resid"], do["op_resid"], dg["op_resid_ramp"], do["op_resid_ramp"])
        assert do["op_resid_ramp"] > 0 and do["op_resid"] < do["op_resid_ramp"]
        assert dg["op_resid"] == pytest.approx(do["op_resid"], rel=tol)
        assert dg["op_resid_ramp"] == pytest.approx(do["op_resid_ramp"], rel=tol)
        if stage == "stepped":
            rg = g.solve_potential(1e-11, 400000)
            ro = o.solve_potential(1e-11, 400000)
            if precision == "fp64":
                assert rg[:2] == ro[:2]


def test_capped_initial_solve_is_reported():
    from paper_2410_06657_amd.lbm import LbmError, Solver
    c = dict(small_drop(1), poisson_max_sweeps=40)
    s = Solver(c)
    assert not s.init_converged and s.diag()["init_converged"] == 0
    assert list(s.sweep_log()) == [40]
    s.step(2)  # the state is valid: the run goes on
    assert s.diag()["nonfinite"] == 0
    with pytest.raises(LbmError):
        Solver(c, require_converged=True)
    ok = Solver(small_drop(1))
    assert ok.init_converged and ok.diag()["init_converged"] == 1


def test_autotune_uses_the_callers_workspace():
    import torch
    from paper_2410_06657_amd import lbm
    c = inputs.scaled(inputs.drop_128x64(3), 192, 96)
    p = lbm.make_params(c, "fp64")
    need = C.c_size_t()
    assert lbm.lib().lbm_autotune_workspace_bytes(C.byref(p), C.byref(need)) == 0
    assert need.value >= lbm.workspace_bytes(c, "fp64")
    stream = torch.cuda.current_stream()
    out = lbm.LbmTune()
    small = torch.empty(need.value - 256, dtype=torch.uint8, device="cuda")
    rc = lbm.lib().lbm_autotune(C.byref(p), C.c_void_p(small.data_ptr()), C.c_size_t(small.numel()),
                                C.c_void_p(stream.cuda_stream), 4, lbm.LBM_TUNE_FORCE, C.byref(out))
    assert rc == lbm.LBM_ESPACE
    ws = torch.full((need.value,), 255, dtype=torch.uint8, device="cuda")
    before = torch.cuda.memory_allocated()
    rc = lbm.lib().lbm_autotune(C.byref(p), C.c_void_p(ws.data_ptr()), need,
                                C.c_void_p(stream.cuda_stream), 4, lbm.LBM_TUNE_FORCE, C.byref(out))
    assert rc == 0 and out.ncand == 6 and out.sweep_block in (2, 4, 8) and out.sweep_waves in (4, 8)
    assert torch.cuda.memory_allocated() == before
    assert int(ws[:4096].ne(255).sum()) > 0  # the candidates' state went into the caller's bytes


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16store"])
def test_field_to_device_equals_host_copy(precision):
    from paper_2410_06657_amd.lbm import FIELDS, Solver
    s = Solver(small_drop(2), precision)
    s.step(3)
    for k in FIELDS:
        d = s.field_device(k).cpu().numpy()
        assert np.array_equal(d, s.field(k)), k


def test_restore_rejects_foreign_or_corrupt_images():
    from paper_2410_06657_amd.lbm import LbmError, Solver
    c = small_drop(5)
    a = Solver(c)
    a.step(2)
    img = bytearray(a.checkpoint())
    b = Solver(c)
    b.restore(bytes(img))  # the image itself is good
    assert np.array_equal(b.field("psi"), a.field("psi"))
    # the header's sp (int32 after magic and six int32 members) and lcur
    for off, val in ((8 + 6 * 4, 5), (8 + 7 * 4, -1)):
        bad = bytearray(img)
        bad[off:off + 4] = int(val).to_bytes(4, "little", signed=True)
        with pytest.raises(LbmError) as e:
            b.restore(bytes(bad))
        assert e.value.code == -1
    other = Solver(dict(c, T_w=c["T_w"] * 1.5))
    with pytest.raises(LbmError) as e:
        other.restore(bytes(img))
    assert e.value.code == -1


def test_checkpoint_refuses_other_stage_rows():
    """The stage segment height is part of the parameter digest: an image restores only into a
    handle with the same value (the fields would not change, but the volume sums' order would)."""
    from paper_2410_06657_amd.lbm import LbmError, Solver
    c = small_drop(6)
    a = Solver(dict(c, stage_rows=8))
    a.step(2)
    img = a.checkpoint()
    with pytest.raises(LbmError) as e:
        Solver(dict(c, stage_rows=16)).restore(img)
    assert e.value.code == -1
    b = Solver(dict(c, stage_rows=8))
    b.restore(img)
    a.step(3)
    b.step(3)
    assert np.array_equal(a.field("psi"), b.field("psi"))


def test_time_copy_copies_and_times():
    """lbm_time_copy moves the bytes it is given (the last of its copies is checked) and reports
    a positive duration."""
    import ctypes as C

    import torch

    from paper_2410_06657_amd import lbm
    n = (64 << 20) + 48  # not a multiple of the 4 x 16-byte pass of a thread
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    ms = C.c_float()
    rc = lbm.lib().lbm_time_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), n,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream), 3, C.byref(ms))
    assert rc == lbm.LBM_OK and ms.value > 0
    assert torch.equal(dst, src)
