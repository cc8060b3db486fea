"""The C-ABI library loads and exports every entry point that include/lbm.h declares
(no compute calls: no GPU here), and the host-side parameter checks work."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def liblbm():
    from paper_2410_06657_amd import build, lbm
    if not os.path.exists(lbm.LIB_PATH):
        build.build()
    return lbm


def declared():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(liblbm):
    names = declared()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_solve_potential" in names
    assert "lbm_diagnostics" in names
    out = subprocess.run(["nm", "-D", "--defined-only", liblbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(lbm_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(liblbm.SYMBOLS) == names


def test_workspace_size_and_validation(liblbm):
    from paper_2410_06657_amd import inputs
    c = inputs.drop_128x64(0)
    n = liblbm.workspace_bytes(c)
    # 66 population planes + 27 field planes of 128 x 64 doubles, plus a small tail
    assert 93 * 128 * 64 * 8 <= n < 93 * 128 * 64 * 8 + 65536
    # FP32: the same planes in floats plus the bases (two sets of 4 potential-link planes, 1
    # enthalpy) and the sweep constants (4 pulled base increments, 1 base potential)
    n32 = liblbm.workspace_bytes(c, "fp32")
    assert 107 * 128 * 64 * 4 <= n32 < 107 * 128 * 64 * 4 + 65536
    # FP16 storage: the 54 planes of f, h and g in binary16, the rest as in FP32
    n16 = liblbm.workspace_bytes(c, "fp16store")
    assert n16 == pytest.approx(n32 - 54 * 128 * 64 * 2, abs=4096)
    big = liblbm.workspace_bytes(inputs.drop_4096x2048())
    assert big > 6e9
    for bad in (dict(c, nx=1), dict(c, ny=2), dict(c, M=0.0), dict(c, sig_l=-1.0),
                dict(c, poisson_max_sweeps=0), dict(c, shape=3), dict(c, sweep_block=3),
                dict(c, sweep_waves=2), dict(c, stage_rows=-4), dict(c, stage_rows=6),
                dict(c, stage_rows=516), dict(c, sweep_block=16), dict(c, sweep_block=16, sweep_waves=4),
                dict(c, sweep_block=32, sweep_waves=8)):
        with pytest.raises(liblbm.LbmError) as e:
            liblbm.workspace_bytes(bad)
        assert e.value.code == liblbm.LBM_EINVAL
    # stage segment rows: any multiple of 4 up to 512 (taller than the grid included)
    for rows in (4, 8, 200, 512):
        assert liblbm.workspace_bytes(dict(c, stage_rows=rows)) > 0
    # the shapes a handle takes, defaults resolved: 32-row segments while the flow launch keeps
    # 2048 workgroups (67 strips of 62 columns at 4096 x 2048), lower on smaller grids
    assert liblbm.launch_shapes(inputs.drop_4096x2048()) == {"sweep_block": 8, "sweep_waves": 4, "stage_rows": 32}
    assert liblbm.launch_shapes(c)["stage_rows"] == 4  # 3 strips x 16 segments at 128 x 64
    assert liblbm.launch_shapes(dict(c, stage_rows=16, sweep_block=4)) == {
        "sweep_block": 4, "sweep_waves": 4, "stage_rows": 16}
    assert liblbm.launch_shapes(dict(c, sweep_block=16, sweep_waves=8))["sweep_block"] == 16


def test_time_copy_argument_checks(liblbm):
    """The copy-bandwidth entry rejects misaligned, odd-sized and overlapping buffers before
    touching the device."""
    import ctypes as C
    L, ms = liblbm.lib(), C.c_float()
    ok_src, ok_dst = C.c_void_p(1 << 20), C.c_void_p(1 << 24)
    assert L.lbm_time_copy(C.c_void_p((1 << 24) + 8), ok_src, 4096, None, 1, C.byref(ms)) == liblbm.LBM_EINVAL
    assert L.lbm_time_copy(ok_dst, ok_src, 4100, None, 1, C.byref(ms)) == liblbm.LBM_EINVAL
    assert L.lbm_time_copy(ok_dst, ok_src, 0, None, 1, C.byref(ms)) == liblbm.LBM_EINVAL
    assert L.lbm_time_copy(ok_dst, ok_src, 4096, None, 0, C.byref(ms)) == liblbm.LBM_EINVAL
    assert L.lbm_time_copy(C.c_void_p((1 << 20) + 2048), ok_src, 4096, None, 1, C.byref(ms)) == liblbm.LBM_EINVAL


def test_error_strings(liblbm):
    L = liblbm.lib()
    for code in range(0, -7, -1):
        assert L.lbm_strerror(code).decode() not in ("", "unknown error")
    assert L.lbm_strerror(-99).decode() == "unknown error"
    # calls on a null handle report a state error instead of crashing
    assert L.lbm_step(None, 1) == liblbm.LBM_ESTATE
    assert L.lbm_destroy(None) == 0


def test_batch_validation(liblbm):
    import ctypes as C
    from paper_2410_06657_amd import inputs
    a = inputs.drop_128x64(0)
    for bad in ([a, dict(a, skip_initial_solve=1)], [a, dict(a, sweep_block=4)], [a, dict(a, sweep_waves=8)]):
        arr = (liblbm.LbmParams * 2)(*[liblbm.make_params(c) for c in bad])
        n = C.c_size_t()
        assert liblbm.lib().lbm_batch_workspace_bytes(2, arr, C.byref(n)) == liblbm.LBM_EINVAL
    # the FP16-storage form batches too (binary16 sets: smaller than the FP32 batch), but every
    # case takes the same precision
    arr = (liblbm.LbmParams * 2)(*[liblbm.make_params(c, "fp16store") for c in (a, a)])
    n16 = C.c_size_t()
    assert liblbm.lib().lbm_batch_workspace_bytes(2, arr, C.byref(n16)) == liblbm.LBM_OK
    arr = (liblbm.LbmParams * 2)(*[liblbm.make_params(c, "fp32") for c in (a, a)])
    n32 = C.c_size_t()
    assert liblbm.lib().lbm_batch_workspace_bytes(2, arr, C.byref(n32)) == liblbm.LBM_OK
    assert n16.value < n32.value
    arr = (liblbm.LbmParams * 2)(liblbm.make_params(a, "fp16store"), liblbm.make_params(a, "fp32"))
    n = C.c_size_t()
    assert liblbm.lib().lbm_batch_workspace_bytes(2, arr, C.byref(n)) == liblbm.LBM_EINVAL
    arr = (liblbm.LbmParams * 2)(*[liblbm.make_params(c) for c in (a, inputs.scaled(a, 64, 32))])
    n = C.c_size_t()
    assert liblbm.lib().lbm_batch_workspace_bytes(2, arr, C.byref(n)) == liblbm.LBM_OK and n.value > 0
