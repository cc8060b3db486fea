"""Pins of the FP64 reference network (oracle/cnn.py): a dilated convolution equals the
library correlation with a dilated kernel, the gradient equals central finite differences,
and the parameter packing round-trips."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def test_param_count_matches_architecture():
    # 3*32*9 + 4*32*32*9 + 32*9 real weights, stored with padded inputs of layer 0
    assert cnn.param_count() == 9 * 32 * 8 + 4 * 9 * 32 * 32 + 9 * 32 * 32 + 6 * 32


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_conv_equals_correlation_with_dilated_kernel(d):
    rng = np.random.default_rng(d)
    a = rng.normal(size=(2, 11, 19, 3))
    w = rng.normal(size=(3, 3, 4, 3))
    b = rng.normal(size=4)
    z = cnn.conv(a, w, b, d)
    for n in range(2):
        for o in range(4):
            ref = np.full((11, 19), b[o])
            for i in range(3):
                k = np.zeros((2 * d + 1, 2 * d + 1))
                k[::d, ::d] = w[:, :, o, i]
                ref += ndimage.correlate(a[n, :, :, i], k, mode="constant", cval=0.0)
            assert np.allclose(z[n, :, :, o], ref, atol=1e-12)


def test_gradient_equals_finite_differences():
    rng = np.random.default_rng(7)
    p = rng.normal(scale=0.15, size=cnn.param_count())
    x = rng.normal(size=(2, 6, 9, 3))
    t = rng.normal(scale=0.3, size=(2, 6, 9))
    loss, g = cnn.loss_and_grad(p, x, t)
    layers = cnn.unpack(p)
    # entries checked: a few real weights of every layer, biases, and padding entries (0)
    off = 0
    picks = []
    for l in range(cnn.NL):
        cs = cnn.CIN_STORED[l]
        for (ky, kx, o, i) in [(0, 0, 0, 0), (1, 1, 0, cnn.CIN_REAL[l] - 1), (2, 1, cnn.COUT_REAL[l] - 1, 1)]:
            picks.append(off + ((3 * ky + kx) * 32 + o) * cs + i)
        off += 9 * 32 * cs
    bias0 = off
    picks += [bias0 + 0, bias0 + 2 * 32 + 5, bias0 + 5 * 32]
    h = 1e-6
    for k in picks:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (cnn.loss_and_grad(pp, x, t)[0] - cnn.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-8), k
    # padding entries: inputs 3..7 of layer 0 and outputs 1..31 of layer 5 do not exist
    assert g[5] == 0.0 and g[4] == 0.0
    last = cnn.param_count() - 6 * 32 - 9 * 32 * 32
    assert g[last + 32 * 1 + 3] == 0.0
    assert loss > 0 and len(layers) == 6


def test_pack_round_trip():
    rng = np.random.default_rng(3)
    p = rng.normal(size=cnn.param_count())
    layers = cnn.unpack(p)
    q = cnn.pack_grad(layers)
    r = cnn.unpack(q)
    for (w1, b1), (w2, b2) in zip(layers, r):
        assert np.array_equal(w1, w2) and np.array_equal(b1, b2)
