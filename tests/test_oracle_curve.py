"""Pins of the oracle's discrete initial curve (section 6.1: a discrete
zero-coupon curve smoothed by splines so that df(0,T)/dT is continuous; the
reading: the natural cubic spline S of -ln P(0,t), f = S', df/dt = S'',
P = exp(-S), constant forward past the last knot).

C1: S, S' and S'' equal scipy's natural cubic spline through the same knots
(an independent implementation) everywhere on the knot range.
C2: the discount reproduces every knot price; S'' is continuous across the
inner knots and zero at both ends, while S''' jumps (a spline, not one cubic).
C3: flat data P = e^{-a t} give f = a and df/dt = 0, and a solve on them
equals the solve on the flat parametric curve.
C4: past the last knot the forward is constant and the discount log-linear,
continuous at the knot.
C5: the bond solved by the scheme reproduces the discrete curve at a knot
maturity at the paper's 1e-5 level, converging at second order in r, with
r0 = f(0,0) taken from scipy's spline.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W


def _problem(seed=4, n=(24, 12, 12)):
    s = W.config_discrete(n, seed)[0]
    return s, to_oracle(s)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_matches_scipy_natural_spline(seed):
    s, p = _problem(seed)
    t, P = np.array(s.model.curve_t), np.array(s.model.curve_p)
    ref = CubicSpline(t, -np.log(P), bc_type="natural")
    for x in np.linspace(0.0, t[-1], 1201)[:-1]:
        assert abs(-math.log(O.discount(p, x)) - ref(x)) <= 1e-13
        assert abs(O.forward(p, x) - ref(x, 1)) <= 1e-13
        assert abs(O.forward_dt(p, x) - ref(x, 2)) <= 1e-13


def test_knots_continuity_and_ends():
    s, p = _problem()
    t, P = np.array(s.model.curve_t), np.array(s.model.curve_p)
    for ti, Pi in zip(t, P):
        assert abs(O.discount(p, ti) - Pi) <= 1e-15 * max(Pi, 1.0)
    eps = 1e-7
    jumps = []
    for ti in t[1:-1]:
        lo, hi = O.forward_dt(p, ti - eps), O.forward_dt(p, ti + eps)
        assert abs(hi - lo) <= 1e-5 * max(abs(hi), 1e-3), ti
        assert abs(O.forward(p, ti + eps) - O.forward(p, ti - eps)) <= 1e-8
        # third derivative on each side, from differences of S''
        d3l = (O.forward_dt(p, ti - eps) - O.forward_dt(p, ti - 1e-3)) / (1e-3 - eps)
        d3r = (O.forward_dt(p, ti + 1e-3) - O.forward_dt(p, ti + eps)) / (1e-3 - eps)
        jumps.append(abs(d3r - d3l))
    assert max(jumps) > 1e-4
    assert abs(O.forward_dt(p, 0.0)) <= 1e-14
    assert abs(O.forward_dt(p, t[-1] - 1e-12)) <= 1e-9


def test_flat_data_is_the_flat_curve():
    a = 0.031
    t = np.array(W.CURVE_KNOTS)
    base = W.config1()[1]
    s_flat = W.with_shape(base, 20, 10, 12, 12)
    p_flat = to_oracle(s_flat)
    p_flat.f_level, p_flat.f_slope, p_flat.f_decay = a, 0.0, 0.0
    p_disc = to_oracle(s_flat)
    p_disc.f_level = 0.0
    p_disc.curve_t, p_disc.curve_p = t, np.exp(-a * t)
    for x in np.linspace(0.0, 25.0, 101):
        assert abs(O.forward(p_disc, x) - a) <= 1e-14
        assert abs(O.forward_dt(p_disc, x)) <= 1e-13
    U_f = O.run(p_flat, 0, p_flat.n_steps)
    U_d = O.run(p_disc, 0, p_disc.n_steps)
    assert np.abs(U_d - U_f).max() <= 1e-13 * np.abs(U_f).max()


def test_extrapolation_past_last_knot():
    s, p = _problem()
    tn = s.model.curve_t[-1]
    f_end = O.forward(p, tn)
    for x in (tn, tn + 0.5, tn + 5.0):
        assert O.forward(p, x) == f_end and O.forward_dt(p, x) == 0.0
    # log-linear and continuous at the knot
    lp = [math.log(O.discount(p, tn + d)) for d in (0.0, 1.0, 2.0)]
    assert abs((lp[0] - lp[1]) - f_end) <= 1e-14 and abs((lp[1] - lp[2]) - f_end) <= 1e-14
    assert abs(math.log(O.discount(p, tn - 1e-9)) - lp[0]) <= 1e-10


def test_bond_reproduces_discrete_curve():
    """Errors of the paper's order (1e-5) that fall at second order with the
    r resolution, as on the parametric sloped curve."""
    ct, cp = W.discrete_curve(4)
    f0 = float(CubicSpline(np.array(ct), -np.log(np.array(cp)), bc_type="natural")(0.0, 1))
    m = W.config_discrete(seed=4)[0].model
    T = 2.0
    errs = []
    for nr in (48, 96):
        s = W.SolveSpec(W.default_axes(nr, 24, 24, f0), m, W.PayoffSpec(W.BOND, T, T + 1.0, 0.03), 80, f0)
        p = to_oracle(s)
        price, _ = O.price(p, s.r0, s.v0)
        errs.append(abs(price - cp[ct.index(T)]))
    assert errs[1] < 2.5e-5, errs
    assert 3.5 < errs[0] / errs[1] < 4.5, errs
