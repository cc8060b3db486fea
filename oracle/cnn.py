"""Plain FP64 reference of the warm-start network (test infrastructure only; never called by
the product path).

Six 3x3 convolutions with zero padding, channels 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1,
dilations 1, 2, 4, 8, 4, 1, tanh after every layer but the last.  Arrays are NHWC.  A
convolution is written out as its definition,

    z[n, y, x, o] = b[o] + sum_{ky, kx, i} a[n, y + (ky - 1) d, x + (kx - 1) d, i] W[ky, kx, o, i],

with a = 0 outside the image, and the gradient of L = sum (y - t)^2 by the chain rule, layer
by layer, in the same notation.  The parameter vector is the library's documented order:
for each layer the weights [tap = 3 ky + kx][out 0..31][in 0..cin-1] (cin = 8 for layer 0,
of which 3 are read; else 32), then 6 x 32 biases; the last layer has one output.
"""
import numpy as np

NL = 6
CH = 32
CIN_STORED = [8, 32, 32, 32, 32, 32]
CIN_REAL = [3, 32, 32, 32, 32, 32]
COUT_REAL = [32, 32, 32, 32, 32, 1]
DIL = [1, 2, 4, 8, 4, 1]


def param_count():
    return sum(9 * CH * c for c in CIN_STORED) + NL * CH


def unpack(p):
    """Parameter vector -> per layer (W[3, 3, cout, cin], b[cout]) with the real sizes."""
    p = np.asarray(p, dtype=np.float64)
    layers = []
    off = 0
    for l in range(NL):
        cs = CIN_STORED[l]
        w = p[off:off + 9 * CH * cs].reshape(3, 3, CH, cs)
        off += 9 * CH * cs
        layers.append(w[:, :, :COUT_REAL[l], :CIN_REAL[l]].copy())
    bias = p[off:off + NL * CH].reshape(NL, CH)
    return [(layers[l], bias[l, :COUT_REAL[l]].copy()) for l in range(NL)]


def pack_grad(grads):
    """Per layer (dW[3, 3, cout, cin], db[cout]) -> vector in parameter order (padding 0)."""
    out = np.zeros(param_count())
    off = 0
    for l in range(NL):
        cs = CIN_STORED[l]
        blk = np.zeros((3, 3, CH, cs))
        dw, _ = grads[l]
        blk[:, :, :COUT_REAL[l], :CIN_REAL[l]] = dw
        out[off:off + 9 * CH * cs] = blk.ravel()
        off += 9 * CH * cs
    for l in range(NL):
        _, db = grads[l]
        out[off + l * CH:off + l * CH + COUT_REAL[l]] = db
    return out


def shifted(a, dy, dx):
    """s[n, y, x, :] = a[n, y + dy, x + dx, :] inside the image, 0 outside."""
    n, h, w, c = a.shape
    s = np.zeros_like(a)
    y0, y1 = max(0, -dy), min(h, h - dy)
    x0, x1 = max(0, -dx), min(w, w - dx)
    if y0 < y1 and x0 < x1:
        s[:, y0:y1, x0:x1, :] = a[:, y0 + dy:y1 + dy, x0 + dx:x1 + dx, :]
    return s


def conv(a, w, b, d):
    """Dilated 3x3 convolution with zero padding (the definition above)."""
    z = np.zeros(a.shape[:3] + (w.shape[2],))
    for ky in range(3):
        for kx in range(3):
            z += shifted(a, (ky - 1) * d, (kx - 1) * d) @ w[ky, kx].T
    return z + b


def forward(p, x):
    """x: (n, h, w, 3) -> y: (n, h, w); also the layer inputs for the backward pass."""
    layers = unpack(p)
    a = np.asarray(x, dtype=np.float64)
    inputs = []
    for l, (w, b) in enumerate(layers):
        inputs.append(a)
        z = conv(a, w, b, DIL[l])
        a = np.tanh(z) if l < NL - 1 else z
    return a[..., 0], inputs


def loss_and_grad(p, x, t):
    """L = sum (y - t)^2 and dL/dp in parameter order."""
    layers = unpack(p)
    y, inputs = forward(p, x)
    e = y - np.asarray(t, dtype=np.float64)
    loss = float(np.sum(e * e))
    dz = (2.0 * e)[..., None]                 # dL/dz of the last layer
    grads = [None] * NL
    for l in range(NL - 1, -1, -1):
        w, _ = layers[l]
        a = inputs[l]
        d = DIL[l]
        dw = np.zeros_like(w)
        for ky in range(3):
            for kx in range(3):
                sa = shifted(a, (ky - 1) * d, (kx - 1) * d)
                dw[ky, kx] = np.einsum("nyxo,nyxi->oi", dz, sa)
        grads[l] = (dw, dz.sum(axis=(0, 1, 2)))
        if l > 0:
            # dL/da[p] = sum over taps of dz[p - offset] W^T, then through tanh of layer l-1
            da = np.zeros_like(a)
            for ky in range(3):
                for kx in range(3):
                    da += shifted(dz @ w[ky, kx], -(ky - 1) * d, -(kx - 1) * d)
            dz = da * (1.0 - a * a)
    return loss, pack_grad(grads)
