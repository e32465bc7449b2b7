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


# ---------------------------------------------------------------------------
# Caplet baseline (the control variate of the surrogate's target)
# ---------------------------------------------------------------------------
import oracle as O  # noqa: E402
from scipy import integrate  # noqa: E402

_CONSTS = (0.15, 0.9, 0.25, 0.5, 1.0)  # lambda, gamma, theta_v, curve decay, tenor


def _gaussian_oracle(x_row, lam_eff, decay=0.5, tenor=1.0):
    """The solver oracle's Gaussian caplet (its own curve, bond and accrual
    code) at the row's strike, with rate volatility lam_eff (gamma = 0)."""
    kap, _, _, _, a, b, dk, T = (float(t) for t in x_row)
    ax = O.Axis(5, 0.0, 1.0, 0.5, 1.0)
    p = O.Problem([ax, ax, ax], kappa=kap, theta_v=0.25, lam=lam_eff, gamma=0.0, epsilon=0.0, rho=0.0,
                  f_level=a, f_slope=b, f_decay=decay, kind=O.CAPLET, expiry=T, pay=T + tenor)
    katm = (O.discount(p, T) / O.discount(p, T + tenor) - 1.0) / tenor
    p.strike = katm + dk
    return O.gaussian_caplet(p)


def test_baseline_gaussian_limit_is_the_closed_form():
    """gamma = 0 and v0 = 1 leave the Gaussian model itself: the baseline must
    be the oracle's textbook caplet (bond put) price."""
    x = M.np.asarray(__import__("paper_1108_1688_amd.workloads", fromlist=["x"]).surrogate_params(12, 7))
    x[:, 3] = 1.0
    x[0, 0] = 0.0  # kappa = 0: G(s) = s, variance factor T
    got = M.caplet_baseline(x, 0.01, 0.0, 0.25, 0.5, 1.0)
    want = np.array([_gaussian_oracle(r, 0.01) for r in x])
    assert np.all(want > 0)
    np.testing.assert_allclose(got, want, rtol=1e-12)


@pytest.mark.parametrize("kappa", [0.05, 0.125, 0.125 + 1e-9, 0.19])
def test_baseline_variance_by_quadrature(kappa):
    """The frozen-volatility variance lam^2 f(0,T)^(2 gamma) G^2 times the
    integral of the variance factor's mean path against e^{-2 kappa (T - t)},
    the integral done by quadrature (kappa = theta_v / 2 is the removable
    singularity of the closed form): with it as an effective Gaussian
    volatility the oracle's closed form must give the same price."""
    lam, gam, thv, dec, ten = _CONSTS
    for v0, T, a, b, dk in ((0.6, 2.5, 0.02, 0.01, 0.004), (1.4, 0.7, 0.035, 0.0, -0.008), (1.0, 4.0, 0.01, 0.02, 0.0)):
        x = np.array([[kappa, 0.3, 0.1, v0, a, b, dk, T]])
        integral, _ = integrate.quad(lambda t: (1.0 + (v0 - 1.0) * math.exp(-thv * t)) * math.exp(-2 * kappa * (T - t)),
                                     0.0, T, epsabs=0, epsrel=1e-13)
        fT = a + b * (1.0 - math.exp(-dec * T))
        var_factor = -math.expm1(-2 * kappa * T) / (2 * kappa)
        lam_eff = lam * fT ** gam * math.sqrt(integral / var_factor)
        got = M.caplet_baseline(x, *_CONSTS)[0]
        np.testing.assert_allclose(got, _gaussian_oracle(x[0], lam_eff), rtol=1e-10)


def test_baseline_bounds_and_strike_order():
    """Between intrinsic value and the expiry bond, decreasing in the strike."""
    x = np.repeat(np.array([[0.1, 0.3, 0.0, 1.0, 0.02, 0.01, 0.0, 2.0]]), 9, axis=0)
    x[:, 6] = np.linspace(-0.01, 0.01, 9)
    B = M.caplet_baseline(x, *_CONSTS)
    assert np.all(np.diff(B) < 0)
    ax = O.Axis(5, 0.0, 1.0, 0.5, 1.0)
    p = O.Problem([ax, ax, ax], kappa=0.1, theta_v=0.25, lam=0.15, gamma=0.9, epsilon=0.3, rho=0.0,
                  f_level=0.02, f_slope=0.01, f_decay=0.5)
    PT, PM = O.discount(p, 2.0), O.discount(p, 3.0)
    K = (PT / PM - 1.0) + x[:, 6]
    assert np.all(B >= np.maximum(PT - (1.0 + K) * PM, 0.0))
    assert np.all(B < PT)


def test_baseline_target_round_trip():
    x = np.random.default_rng(3).random((7, 8)) * 0.0 + np.array([0.1, 0.3, 0.0, 1.0, 0.02, 0.01, 0.001, 1.5])
    price = np.linspace(1e-4, 5e-3, 7)
    t = M.baseline_target(x, price, 0.1, 0.0, _CONSTS)
    np.testing.assert_allclose(M.baseline_price(x, t, 0.1, 0.0, _CONSTS), price, rtol=1e-13)
