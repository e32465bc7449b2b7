"""CPU oracle of the surrogate MLP (8 -> 256 -> 256 -> 256 -> 256 -> 1, GELU).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product never does.  Plain numpy, no
code shared with the HIP path.

Modes:
  exact    every quantity in float64 (pinned by finite differences);
  emulate  the GPU's rounding points: inputs normalised in float32 and rounded
           to BF16, weights rounded from the FP32 masters to BF16, every
           hidden activation GELU(Z) rounded to BF16, the back-propagated
           dZ rounded to BF16; products and sums of those BF16 values in
           float64;
  emulate32  as emulate, with the layer sums Z accumulated in float32 (in
           numpy's order, not the GPU's): its distance from emulate measures
           how much the accumulation order alone moves the BF16 roundings.

Caplet baseline (control variate of the network's target): the Gaussian
(Hull-White) caplet price, the zero-coupon bond put of the textbook model,
with the rate volatility frozen at lambda f(0,T)^gamma times the root of the
variance factor's mean path v(t) = 1 + (v0 - 1) e^{-theta_v t} (the mean of
the paper's section 3.1 variance process).  Written from the model's
definitions; pinned against the solver oracle's Gaussian closed form (gamma =
0, v0 = 1) and against quadrature of the variance integral.

The loss is the mean squared error in network units, L = mean((y - t)^2); the
optimiser is Adam (Kingma and Ba, "Adam: a method for stochastic
optimization", Algorithm 1), with bias-corrected first and second moments.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN = 8
HID = 256
# flat parameter layout: W1 (256 x 8), b1, W2 (256 x 256), b2, W3, b3, W4, b4, w5, b5
SHAPES = [("W1", (HID, N_IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, HID)), ("b4", (HID,)),
          ("w5", (HID,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 199,937


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    assert o == N_PARAMS
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round float32 values to BF16 (8 significant bits), nearest, ties to
    even; returned as float64 holding the BF16 value."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    """GELU(z) = z Phi(z), Phi the standard normal distribution function."""
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_d(z):
    """d/dz GELU(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def normalise(x, lo, hi, emulate: bool):
    """Map each input to [-1, 1] over the box; returns (inputs, in_box)."""
    if emulate:
        x32 = np.asarray(x, dtype=np.float32)
        lo32 = np.asarray(lo, dtype=np.float32)
        hi32 = np.asarray(hi, dtype=np.float32)
        inside = np.all((x32 >= lo32) & (x32 <= hi32), axis=1)
        z = np.float32(2.0) * (x32 - lo32) / (hi32 - lo32) - np.float32(1.0)
        return bf16(z), inside
    x = np.asarray(x, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    inside = np.all((x >= lo) & (x <= hi), axis=1)
    return 2.0 * (x - lo) / (hi - lo) - 1.0, inside


def _weights(P: dict, emulate: bool) -> dict:
    if not emulate:
        return P
    W = dict(P)
    for name in ("W1", "W2", "W3", "W4", "w5"):
        W[name] = bf16(P[name])
    return W


def forward(p, x, lo, hi, emulate=True):
    """Network output (network units) and the cache for the backward pass;
    emulate is False, True or "emulate32"."""
    P = unpack(np.asarray(p, dtype=np.float64))
    acc32 = emulate == "emulate32"
    emulate = bool(emulate)
    W = _weights(P, emulate)
    h, inside = normalise(x, lo, hi, emulate)
    hs, zs = [h], []
    for l in (1, 2, 3, 4):
        if acc32:
            z = (hs[-1].astype(np.float32) @ W[f"W{l}"].T.astype(np.float32)).astype(np.float64)
            z = (z.astype(np.float32) + np.asarray(P[f"b{l}"], dtype=np.float32)).astype(np.float64)
        else:
            z = hs[-1] @ W[f"W{l}"].T + np.asarray(P[f"b{l}"], dtype=np.float32 if emulate else np.float64)
        a = gelu(z)
        zs.append(z)
        hs.append(bf16(a) if emulate else a)
    y = hs[-1] @ W["w5"] + P["b5"][0]
    return y, {"hs": hs, "zs": zs, "W": W, "inside": inside}


def loss_and_grads(p, x, t, lo, hi, emulate: bool = True):
    """Summed squared error and the gradient of the mean squared error."""
    y, c = forward(p, x, lo, hi, emulate)
    n = len(t)
    e = y - np.asarray(t, dtype=np.float64)
    dy = 2.0 * e / n
    W, hs, zs = c["W"], c["hs"], c["zs"]
    g = {"w5": hs[4].T @ dy, "b5": np.array([dy.sum()])}
    dz = dy[:, None] * W["w5"][None, :] * gelu_d(zs[3])
    if emulate:
        dz = bf16(dz)
    for l in (4, 3, 2, 1):
        g[f"W{l}"] = dz.T @ hs[l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        if l > 1:
            dh = dz @ W[f"W{l}"]
            dz = dh * gelu_d(zs[l - 2])
            if emulate:
                dz = bf16(dz)
    return float(e @ e), pack(g)


def adam_step(p, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step count t >= 1); returns the new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def _ndtr(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0)))


def caplet_baseline(x, lam, gam, theta_v, decay, tenor):
    """Gaussian caplet price of each row (kappa, eps, rho, v0, level, slope,
    strike offset, expiry): the curve f(0,t) = level + slope (1 - e^{-decay t}),
    payment one tenor after expiry, strike = at-the-money (simple
    compounding over the tenor) + offset.  Returns float64 prices."""
    x = np.asarray(x, dtype=np.float64)
    kap, v0, a, b, dk, T = x[:, 0], x[:, 3], x[:, 4], x[:, 5], x[:, 6], x[:, 7]
    TM = T + tenor

    def int_f(t):  # integral of f(0, s) over [0, t]
        return a * t + b * (t - (1.0 - np.exp(-decay * t)) / decay)

    PT, PM = np.exp(-int_f(T)), np.exp(-int_f(TM))
    K = (PT / PM - 1.0) / tenor + dk
    D = 1.0 + tenor * K
    G = np.where(kap > 0, -np.expm1(-kap * tenor) / np.where(kap > 0, kap, 1.0), tenor)
    fT = a + b * (1.0 - np.exp(-decay * T))
    # variance of ln P(T, T_M) at expiry: lam^2 fT^(2 gam) G^2 int_0^T vbar(t) e^{-2 kap (T - t)} dt
    I1 = np.where(kap > 0, -np.expm1(-2.0 * kap * T) / np.where(kap > 0, 2.0 * kap, 1.0), T)
    d = 2.0 * kap - theta_v
    # (e^{-theta_v T} - e^{-2 kap T}) / d without the cancellation near d = 0
    I2 = np.exp(-2.0 * kap * T) * np.where(d != 0, np.expm1(d * T) / np.where(d != 0, d, 1.0), T)
    var = lam ** 2 * fT ** (2.0 * gam) * G ** 2 * (I1 + (v0 - 1.0) * I2)
    s = np.sqrt(var)
    h = np.log(D * PM / PT) / s + 0.5 * s
    return PT * _ndtr(s - h) - D * PM * _ndtr(-h)


def baseline_target(x, price, scale, shift, consts):
    """Network target of a price with the baseline: (ln(price / B) - shift) / scale."""
    B = caplet_baseline(x, *consts)
    return (np.log(np.asarray(price, dtype=np.float64) / B) - shift) / scale


def baseline_price(x, y, scale, shift, consts):
    """Price from the network output y: B exp(y scale + shift)."""
    return caplet_baseline(x, *consts) * np.exp(np.asarray(y, dtype=np.float64) * scale + shift)
