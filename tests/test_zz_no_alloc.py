"""The allocation-free forward pass of the warm-start network (lbm_nn_forward_noalloc) against
lbm_nn_forward, through the C ABI: bitwise equal outputs on two calls in a row, the second with
a smaller input; sizes beyond the scratch are refused on the host; no device memory is
allocated by the call."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(net, x, y):
    from paper_2410_06657_amd import lbm
    L = lbm.lib()
    L.lbm_nn_forward_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int]
    n, h, w = net._shape(x)
    return L.lbm_nn_forward_noalloc(net._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), n, h, w)


def test_noalloc_forward_equals_forward():
    import torch
    from paper_2410_06657_amd import warm
    from paper_2410_06657_amd.lbm import Net
    print("no-alloc forward: 2x32x128 then 1x24x40 pixels", flush=True)
    net = Net(8192, seed=3)
    net.set_params(np.load(warm.WEIGHTS).astype(np.float32))
    g = torch.Generator(device="cuda").manual_seed(11)
    for shape in ((2, 32, 128, 3), (1, 24, 40, 3)):
        x = torch.randn(shape, generator=g, device="cuda", dtype=torch.float32)
        ref = net.forward(x)
        torch.cuda.synchronize()
        y = torch.full(shape[:3], float("nan"), device="cuda", dtype=torch.float32)
        before = torch.cuda.memory_allocated()
        assert _noalloc(net, x, y) == 0
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(y, ref), shape
        assert torch.isfinite(y).all()
    big = torch.zeros((1, 128, 129, 3), device="cuda")
    out = torch.zeros((1, 128, 129), device="cuda")
    assert _noalloc(net, big, out) == -1  # beyond the scratch: refused before any launch
