"""Pins of the surrogate MLP's CPU oracle against mathematics, not itself:
central finite differences of the float64 network, the GELU definition and
its derivative, BF16 rounding on values whose rounding is known, Adam's first
step, and a network whose output is known in closed form."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    P = {}
    for name, shape in M.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else M.HID
        P[name] = rng.standard_normal(shape) * (scale / math.sqrt(fan_in) if len(shape) == 2 else 0.1)
    P["w5"] = rng.standard_normal(M.HID) / math.sqrt(M.HID)
    return M.pack(P)


def _data(seed, n):
    rng = np.random.default_rng(seed)
    lo, hi = -np.ones(8), 2 * np.ones(8)
    x = lo + (hi - lo) * rng.random((n, 8))
    t = rng.standard_normal(n)
    return x, t, lo, hi


def test_parameter_count():
    assert M.N_PARAMS == 199937


def test_gradient_matches_central_differences_in_float64():
    p = _params(1)
    x, t, lo, hi = _data(2, 5)
    _, g = M.loss_and_grads(p, x, t, lo, hi, emulate=False)
    rng = np.random.default_rng(3)
    # every bias and output weight plus a sample of each weight matrix
    idx = list(range(2048, 2304)) + list(rng.choice(2048, 40, replace=False))
    o = 2304
    for _ in range(3):
        idx += list(o + rng.choice(65536, 40, replace=False)) + list(range(o + 65536, o + 65536 + 256, 7))
        o += 65536 + 256
    idx += list(range(o, o + 257, 3))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = M.loss_and_grads(pp, x, t, lo, hi, emulate=False)
        lm, _ = M.loss_and_grads(pm, x, t, lo, hi, emulate=False)
        fd = (lp - lm) / (2 * h) / len(t)  # loss_and_grads returns the summed error
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_gelu_definition_and_derivative():
    z = np.linspace(-6, 6, 241)
    Phi = np.array([0.5 * (1 + math.erf(v / math.sqrt(2))) for v in z])
    assert np.allclose(M.gelu(z), z * Phi, rtol=0, atol=1e-15)
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15  # Phi(1)
    h = 1e-5
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_d(z), fd, atol=1e-9)


def test_bf16_rounding():
    one = 1.0
    ulp = 2.0 ** -7  # spacing of BF16 numbers in [1, 2)
    cases = {one: one, one + ulp: one + ulp, one + ulp / 2: one,  # tie to even
             one + 1.5 * ulp: one + 2 * ulp,  # tie to even (upward)
             one + 0.75 * ulp: one + ulp, -3.0: -3.0, 0.0: 0.0}
    for x, want in cases.items():
        assert M.bf16(np.float32(x))[()] == want, x
    r = np.random.default_rng(0).standard_normal(1000)
    b = M.bf16(r)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2.0 ** -8 * (1 + 1e-6))


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3])
    p1, m, v = M.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_known_network_output():
    # W1 picks input 0 (normalised to [-1, 1]) into unit 0, all else zero:
    # h1 = GELU(x0n), h2 = GELU(GELU(x0n)), ..., y = 2 GELU^4(x0n) + 0.5
    P = {name: np.zeros(shape) for name, shape in M.SHAPES}
    P["W1"][0, 0] = 1.0
    for l in (2, 3, 4):
        P[f"W{l}"][0, 0] = 1.0
    P["w5"][0] = 2.0
    P["b5"][0] = 0.5
    x, _, lo, hi = _data(5, 16)
    y, c = M.forward(M.pack(P), x, lo, hi, emulate=False)
    xn = 2 * (x[:, 0] - lo[0]) / (hi[0] - lo[0]) - 1
    want = 2 * M.gelu(M.gelu(M.gelu(M.gelu(xn)))) + 0.5
    assert np.allclose(y, want, rtol=0, atol=1e-14)
    assert c["inside"].all()
    x2 = x.copy()
    x2[3, 5] = hi[5] + 1e-3
    _, c2 = M.forward(M.pack(P), x2, lo, hi, emulate=True)
    assert not c2["inside"][3] and c2["inside"].sum() == 15


def test_emulated_forward_is_close_to_exact():
    p = _params(7)
    x, t, lo, hi = _data(8, 64)
    ye, _ = M.forward(p, x, lo, hi, emulate=True)
    yx, _ = M.forward(p, x, lo, hi, emulate=False)
    assert np.abs(ye - yx).max() < 0.05 * np.abs(yx).max()
