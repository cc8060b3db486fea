"""Training of the warm-start network on potentials the method itself produces.

Samples: single sessile drops on 256 x 128 grids with random size, position, contact angle,
conductivity ratio R and permittivity ratio S (plus drops deformed by a strong field for a few
hundred steps), their potentials solved by the library's own sweeps to a relative change of
1e-9 in FP64 (the batched form runs 96 cases per launch), reduced by the library's coarse-map
kernels with factor 4 to 32 x 64 maps.  The network sees coarse maps of fixed aspect and
resolution (ny / factor = 32 rows), so a grid of height ny is warm-started with factor ny / 32.

Training: Adam on L = sum (y - t)^2 with the library's forward/backward/update kernels,
minibatches of 64 random samples, random periodic x shifts and mirror images (both exact
symmetries of the potential problem), cosine learning-rate decay.

    python -m paper_2410_06657_amd.warm --samples 16000 --iters 20000 --out <path>.npy
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "warm_start_net.npy")
COARSE_ROWS = 32


def factor_for(ny: int) -> int:
    """Coarsening factor that maps a grid of height ny to the network's 32 coarse rows."""
    if ny % COARSE_ROWS:
        raise ValueError(f"ny = {ny} is not a multiple of {COARSE_ROWS}")
    return ny // COARSE_ROWS


def coarse_factor(nx: int, ny: int, rows: int = COARSE_ROWS) -> int:
    """The common divisor f of nx and ny that gives ny / f nearest `rows` coarse rows (ties: the
    larger f); the rule lbm_batch_warm_start applies to every case of a batch."""
    best, err = 1, float("inf")
    for f in range(1, ny + 1):
        if nx % f or ny % f:
            continue
        e = abs(ny / f - rows)
        if e <= err:
            best, err = f, e
    return best


def training_cases(rng, count: int, ny: int = 128, deformed: bool = False) -> list:
    from . import inputs
    cases = []
    for _ in range(count):
        R0 = rng.uniform(0.12, 0.42) * ny
        theta = rng.uniform(45.0, 135.0)
        R = math.exp(rng.uniform(math.log(0.2), math.log(8.0)))
        S = math.exp(rng.uniform(math.log(0.5), math.log(3.0)))
        Ca = rng.uniform(0.5, 1.5) if deformed else 0.1
        c = inputs.sessile_drop(2 * ny, ny, R0, theta, R, S, Ca, 0.1, seed=int(rng.integers(1 << 62)))
        c["xc"] = rng.uniform(0.0, 2 * ny)
        # no freezing while a deformed shape develops
        if deformed:
            c.update(T_w=0.05, T_g=0.05)
        c.update(poisson_tol=1e-9, poisson_max_sweeps=400000)
        cases.append(c)
    return cases


def make_dataset(nsamples: int, seed: int = 5, ny: int = 128, log=print):
    """(x, t): torch FP32 device tensors (n, 32, 64, 3) and (n, 32, 64)."""
    import torch

    from .lbm import Batch

    f = factor_for(ny)
    rng = np.random.default_rng(seed)
    xs, ts = [], []
    k = 0
    t0 = time.time()
    while k < nsamples:
        nb = min(96, nsamples - k)
        deformed = (k // 96) % 3 == 2
        cases = training_cases(rng, nb, ny, deformed)
        b = Batch(cases, precision="fp64")
        if deformed:
            b.step(int(rng.integers(100, 300)))
        for c in range(nb):
            x, t = b.nn_sample(c, f)
            if bool(torch.isfinite(x).all()) and bool(torch.isfinite(t).all()):
                xs.append(x)
                ts.append(t)
        del b
        k += nb
        log(f"[warm] samples {k}/{nsamples} ({time.time() - t0:.0f}s)")
    return torch.stack(xs), torch.stack(ts)


def train(x, t, iters: int = 20000, batch: int = 64, lr: float = 2e-3, seed: int = 1, log=print,
          holdout: int = 512):
    """Train a fresh network; returns (net, history)."""
    import torch

    from .lbm import Net

    n, h, w, _ = x.shape
    gen = torch.Generator(device="cpu").manual_seed(seed)
    ntr = n - holdout
    net = Net(batch * h * w, seed=seed)
    hist = []
    t0 = time.time()
    for it in range(iters):
        idx = torch.randint(0, ntr, (batch,), generator=gen)
        shift = int(torch.randint(0, w, (1,), generator=gen))
        flip = bool(torch.randint(0, 2, (1,), generator=gen))
        xb, tb = x[idx.to(x.device)], t[idx.to(x.device)]
        xb, tb = torch.roll(xb, shift, dims=2), torch.roll(tb, shift, dims=2)
        if flip:
            xb, tb = torch.flip(xb, dims=[2]), torch.flip(tb, dims=[2])
        rate = 1e-4 + 0.5 * (lr - 1e-4) * (1 + math.cos(math.pi * it / iters))
        want = it % 1000 == 0 or it == iters - 1
        loss = net.train_step(xb, tb, rate, want_loss=want)
        if want:
            hist.append((it, loss / (batch * h * w)))
            log(f"[warm] iter {it} lr {rate:.2e} mse {loss / (batch * h * w):.3e} ({time.time() - t0:.0f}s)")
    return net, hist


def holdout_error(net, x, t, holdout: int = 512):
    """Relative L2 error of the prediction on the held-out samples (the last `holdout`)."""
    n = x.shape[0]
    num = den = 0.0
    for a in range(n - holdout, n, 64):
        tb = t[a:a + 64]
        y = net.forward(x[a:a + 64])
        num += float((y - tb).pow(2).sum())
        den += float(tb.pow(2).sum())
    return math.sqrt(num / max(den, 1e-30))


def load(max_pixels: int, path: str = WEIGHTS, device: str = "cuda:0"):
    """A network with the committed (or given) trained parameters."""
    from .lbm import Net
    net = Net(max_pixels, device=device)
    net.set_params(np.load(path, allow_pickle=False))
    return net


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--samples", type=int, default=16000)
    ap.add_argument("--iters", type=int, default=20000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--holdout", type=int, default=512)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    x, t = make_dataset(args.samples, log=log)
    net, hist = train(x, t, iters=args.iters, lr=args.lr, log=log, holdout=args.holdout)
    err = holdout_error(net, x, t, args.holdout)
    log(f"[warm] held-out relative L2 error of the coarse potential deviation: {err:.4f}")
    np.save(args.out, net.params(), allow_pickle=False)
    log(f"[warm] wrote {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
