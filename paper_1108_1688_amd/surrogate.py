"""Learned surrogate of the caplet price, trained on the Douglas-ADI solver.

Workflow (each step runs in the library's kernels; this module only moves
arguments):
  training_set   ADI solves at 64^3 (batched), 16 readouts v0 per solve;
  init_params    seeded initial weights (an input of the training, so that a
                 reference computation can start from the same point);
  fit            epochs of shuffled minibatches (GPU forward, backward, Adam);
  price          surrogate inside the training box, ADI outside it.

Inputs per row: kappa, epsilon, rho, v0, curve level, curve slope, strike
offset from the at-the-money strike, expiry (the caplet pays one year after
expiry).  The network predicts ln(price / B) / OUT_SCALE, B the Gaussian
caplet baseline of the library (a control variate computed on the device:
the textbook Gaussian caplet at a frozen effective volatility), so that the
squared-error loss weighs relative errors; make_mlp(baseline=False) gives
the plain network that predicts price / PLAIN_SCALE.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import hjm
from . import workloads as W

OUT_SCALE = 0.1     # network units with the baseline: 10 ln(price / B)
PLAIN_SCALE = 1e-3  # network units without it: prices in units of 1e-3
# the baseline's model constants: lambda, gamma, theta_v (section 3.3 values of
# the solves), curve decay and tenor of the training rows
GAUSS_ARGS = (W.LAMBDA, W.GAMMA, W.THETA_V, W.SURROGATE_F_DECAY, W.SURROGATE_TENOR)
# rows priced at or below this are left out of the training (log target): the
# relative error is stated above it, and the deep out-of-the-money rows below
# it stretch the log-ratio's range (to 97 from 29), which the BF16
# activations' rounding then turns into error on every row
FIT_PRICE_FLOOR = 1e-4
SOFTEN = 0          # terminal data of the solves the network learns from and is checked against


def init_params(seed: int) -> np.ndarray:
    """Seeded initial parameters: weights N(0, 2 / fan_in), biases zero
    (fan-in scaling for GELU layers); the output layer N(0, 1 / 256)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((256, 8), (256, 256), (256, 256), (256, 256)):
        parts.append(rng.standard_normal((fan_out, fan_in)).ravel() * math.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    parts.append(rng.standard_normal(256) / 16.0)
    parts.append(np.zeros(1))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == hjm.MLP_PARAMS
    return p


def training_set(n_solves: int, seed: int, n: int = W.SURROGATE_N, chunk: int = 256, stream=None,
                 soften: int = SOFTEN, readouts: int = 16):
    """Inputs (n_solves * readouts, 8) float32 and ADI prices (float64): every
    solve is read out at `readouts` values of v0 (W.surrogate_readouts: the
    16-point grid, or seeded draws)."""
    params = W.surrogate_params(n_solves, seed)
    v0s = W.surrogate_readouts(n_solves, readouts, seed + 1)
    xs, ps = [], []
    for c0 in range(0, n_solves, chunk):
        rows = params[c0:c0 + chunk]
        specs = [W.surrogate_solve(x, n, soften) for x in rows]
        b = hjm.Batch(specs, stream=stream)
        b.run()
        r0 = np.array([s.r0 for s in specs])
        for q in range(readouts):
            v0 = v0s[c0:c0 + chunk, q]
            prices = b.prices(r0, v0)
            x = rows.copy()
            x[:, 3] = v0
            xs.append(x)
            ps.append(prices)
        b.close()
    return np.concatenate(xs).astype(np.float32), np.concatenate(ps)


def adi_prices(x: np.ndarray, n: int = W.SURROGATE_N, chunk: int = 256, stream=None,
               soften: int = SOFTEN) -> np.ndarray:
    """Reference prices of arbitrary rows by the ADI solver (one solve per row)."""
    out = np.empty(len(x))
    for c0 in range(0, len(x), chunk):
        rows = x[c0:c0 + chunk]
        specs = [W.surrogate_solve(r, n, soften) for r in rows]
        b = hjm.Batch(specs, stream=stream)
        b.run()
        out[c0:c0 + chunk] = b.prices()
        b.close()
    return out


def make_mlp(max_batch: int = 65536, stream=None, baseline: bool = True) -> hjm.Mlp:
    if not baseline:
        return hjm.Mlp(W.SURROGATE_BOX_LO, W.SURROGATE_BOX_HI, PLAIN_SCALE, 0.0, max_batch=max_batch, stream=stream)
    m = hjm.Mlp(W.SURROGATE_BOX_LO, W.SURROGATE_BOX_HI, OUT_SCALE, 0.0, max_batch=max_batch, stream=stream)
    m.set_baseline(*GAUSS_ARGS)
    return m


@dataclass
class FitResult:
    losses: list
    seconds: float


def fit(mlp: hjm.Mlp, x: np.ndarray, prices: np.ndarray, epochs: int, batch: int = 1024, lr: float = 1e-3,
        lr_final: Optional[float] = None, seed: int = 0) -> FitResult:
    """Train on (x, prices): the targets come from the library
    (hjm_mlp_targets; with the baseline, rows priced at or below
    FIT_PRICE_FLOOR are left out); per epoch the rows are shuffled (seeded) on
    the host and one GPU pass over minibatches runs; the learning rate decays
    geometrically from lr to lr_final."""
    import torch
    dev = mlp.device
    if mlp.baseline is not None:
        keep = np.asarray(prices) > FIT_PRICE_FLOOR
        x, prices = np.asarray(x)[keep], np.asarray(prices)[keep]
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    pd = torch.from_numpy(np.ascontiguousarray(prices, dtype=np.float64)).to(dev)
    td = mlp.targets(xd, pd)
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        rate = lr if lr_final is None or epochs == 1 else lr * (lr_final / lr) ** (ep / (epochs - 1))
        perm = torch.from_numpy(rng.permutation(len(x))).to(dev)
        xe = xd.index_select(0, perm).contiguous()
        te = td.index_select(0, perm).contiguous()
        losses.append(mlp.train_epoch(xe, te, batch, rate))
    torch.cuda.synchronize(dev)
    return FitResult(losses, time.perf_counter() - t0)


@dataclass
class Priced:
    prices: np.ndarray     # float64
    in_box: np.ndarray     # bool
    n_fallback: int


def price(mlp: hjm.Mlp, x: np.ndarray, n: int = W.SURROGATE_N, stream=None, soften: int = SOFTEN) -> Priced:
    """Surrogate prices inside the training box, ADI prices outside it."""
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(mlp.device)
    y, inb = mlp.infer(xd)
    out = y.double().cpu().numpy()
    inside = inb.cpu().numpy().astype(bool)
    outside = np.nonzero(~inside)[0]
    if len(outside):
        out[outside] = adi_prices(x[outside].astype(np.float64), n=n, stream=stream, soften=soften)
    return Priced(out, inside, len(outside))


def main(argv=None) -> None:
    """Train a surrogate on a small ADI set, then run in-box inference
    repeatedly and print the times (a short run to trace with a profiler)."""
    import argparse
    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--train-solves", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--infer-rows", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    x, prices = training_set(a.train_solves, seed=21)
    m = make_mlp(max_batch=max(a.infer_rows, 1024))
    m.set_params(init_params(22))
    fr = fit(m, x, prices, epochs=a.epochs, batch=1024, lr=2e-3, lr_final=1e-4, seed=23)
    print(f"surrogate: {len(x)} rows, {a.epochs} epochs in {fr.seconds:.2f} s, final loss {fr.losses[-1]:.3e}",
          flush=True)
    xq = torch.from_numpy(W.surrogate_params(a.infer_rows, seed=24).astype(np.float32)).to(m.device)
    m.infer(xq)
    torch.cuda.synchronize(m.device)
    t0 = time.perf_counter()
    for _ in range(a.reps):
        m.infer(xq)
    torch.cuda.synchronize(m.device)
    el = (time.perf_counter() - t0) / a.reps
    print(f"surrogate: inference of {a.infer_rows} rows in {el * 1e6:.1f} us per pass", flush=True)
    m.close()


if __name__ == "__main__":
    main()
