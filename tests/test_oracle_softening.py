"""Pins of the oracle's softened terminal data (section 7.2: the payoff
averaged over each node's control element).

F1: the Gauss-Legendre rule equals numpy's (leggauss) and integrates
polynomials up to degree 2n - 1 exactly.
F2: each cell average equals a brute-force double integral of the pointwise
payoff (scipy dblquad) over the same rectangle, on cells across the kink,
in the money and out of the money, for caplet, floorlet, forward and bond,
within the y rule's error (5e-9 relative).
F3: the softened terminal grid holds, at each node, the average over its
element centred in the mesh coordinates (every non-Dirichlet node, or only
where the kink crosses the element), keeps the pointwise data elsewhere, and
averages over a partition of a rectangle add up to the integral over it.
F4: on short elements (the r integral of e^{-G r} over an element of width
1e-4..1e-2, where a difference of two exponentials would lose digits) the
average equals a 40-digit evaluation of the same y rule to a few units in
the last place of the payoff's O(1) terms.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W


def test_gauss_legendre_rule():
    x, w = O.gauss_legendre(16)
    xr, wr = np.polynomial.legendre.leggauss(16)
    order = np.argsort(x)
    assert np.allclose(x[order], xr, atol=1e-15) and np.allclose(w[order], wr, atol=1e-15)
    for deg in range(32):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-14, deg


def _problem(kind):
    s = W.config1()[1]
    p = to_oracle(s)
    p.kind = kind
    return p


def _brute(p, rlo, rhi, ylo, yhi):
    val, _ = integrate.dblquad(lambda y, r: O.payoff(p, r, y), rlo, rhi, ylo, yhi, epsabs=1e-14, epsrel=1e-12)
    return val / ((rhi - rlo) * (yhi - ylo))


@pytest.mark.parametrize("kind", [W.CAPLET, W.FLOORLET, W.FORWARD, W.BOND])
def test_cell_average_equals_double_integral(kind):
    p = _problem(kind)
    # the kink of the 1y caplet near r ~ 3 %: cells across it, below, above
    cells = [(0.025, 0.036, 0.0, 0.004), (0.030, 0.031, 0.001, 0.0025), (0.0, 0.01, 0.0, 0.02),
             (0.2, 0.35, 0.005, 0.025), (0.0301, 0.0309, 0.0, 0.025)]
    for rlo, rhi, ylo, yhi in cells:
        got = O.payoff_cell(p, rlo, rhi, ylo, yhi)
        want = _brute(p, rlo, rhi, ylo, yhi)
        # the y rule (16 Gauss-Legendre points) meets an integrand with a
        # jump in its second derivative where the kink leaves the r interval:
        # measured 1.2e-9 relative there, 1e-11 elsewhere
        assert abs(got - want) <= 5e-9 * max(abs(want), 1e-3), (kind, (rlo, rhi, ylo, yhi), got, want)


def _zmap(ax, x):
    c1 = math.asinh((ax.z_min - ax.center) / ax.alpha)
    c2 = math.asinh((ax.z_max - ax.center) / ax.alpha)
    return ax.center + ax.alpha * math.sinh(c2 * x + c1 * (1.0 - x))


@pytest.mark.parametrize("mode", [1, 2])
def test_terminal_grid_softened(mode):
    """Every non-Dirichlet node (mode 1), or the nodes whose element the kink
    crosses (mode 2), takes the average over its element [z(x - h/2),
    z(x + h/2)] in r and y (the map written out here); Dirichlet nodes and,
    in mode 2, nodes away from the kink keep the pointwise data."""
    s = W.with_shape(W.config1()[1], 24, 6, 12, 10)
    p = to_oracle(s)
    U0 = O.terminal(p)
    p.soften = mode
    U1 = O.terminal(p)
    ar, ay = p.axes[0], p.axes[2]
    nr, ny = ar.n, ay.n
    assert np.array_equal(U1[:, :, -1], U0[:, :, -1]) and np.array_equal(U1[-1], U0[-1])
    assert np.all(U1 == U1[:, :1, :])
    changed = 0
    for k in range(ny - 1):
        for i in range(nr - 1):
            rlo, rhi = _zmap(ar, (i - 0.5) / (nr - 1)), _zmap(ar, (i + 0.5) / (nr - 1))
            ylo, yhi = _zmap(ay, (k - 0.5) / (ny - 1)), _zmap(ay, (k + 0.5) / (ny - 1))
            avg = O.payoff_cell(p, rlo, rhi, ylo, yhi)
            crosses = min(O.payoff(p, rlo, ylo), O.payoff(p, rlo, yhi)) == 0.0 < max(O.payoff(p, rhi, ylo),
                                                                                        O.payoff(p, rhi, yhi))
            if mode == 1 or crosses:
                # the map written out here may differ from the oracle's in the last bit
                assert abs(U1[k, 0, i] - avg) <= 1e-12 * max(abs(avg), 1e-3), (k, i, U1[k, 0, i], avg)
                changed += U1[k, 0, i] != U0[k, 0, i]
            else:
                assert U1[k, 0, i] == U0[k, 0, i], (k, i)
    assert changed >= ny - 1


def test_partition_of_averages_is_the_integral():
    """Averages over elements that tile a rectangle add up, weighted by their
    areas, to the payoff's integral over it."""
    p = _problem(W.CAPLET)
    ar, ay = p.axes[0], p.axes[2]
    xr = np.linspace(0.2, 0.5, 13)
    xy = np.linspace(0.0, 0.6, 7)
    rb = [_zmap(ar, x) for x in xr]
    yb = [_zmap(ay, x) for x in xy]
    total = sum((rb[i + 1] - rb[i]) * (yb[k + 1] - yb[k]) * O.payoff_cell(p, rb[i], rb[i + 1], yb[k], yb[k + 1])
                for i in range(len(rb) - 1) for k in range(len(yb) - 1))
    want, _ = integrate.dblquad(lambda yy, rr: O.payoff(p, rr, yy), rb[0], rb[-1], yb[0], yb[-1],
                                epsabs=1e-15, epsrel=1e-12)
    assert abs(total - want) <= 5e-9 * abs(want), (total, want)


@pytest.mark.parametrize("kind", [W.CAPLET, W.FLOORLET, W.FORWARD])
def test_short_elements_keep_their_digits(kind):
    mp = pytest.importorskip("mpmath")
    p = _problem(kind)
    G = -math.expm1(-p.kappa * (p.pay - p.expiry)) / p.kappa
    # c = Delta p(0,T_M)/p(0,T) e^{G f(0,T)}: the forward's pointwise payoff at r = 0, y = 0 is 1 - c
    c = 1.0 - O.payoff(_problem(W.FORWARD), 0.0, 0.0)
    xq, wq = O.gauss_legendre(16)
    mp.mp.dps = 40
    Gm, cm = mp.mpf(G), mp.mpf(c)
    worst = 0.0
    for rlo in (0.0, 0.02, 0.029, 0.031, 0.05):
        for width in (1e-4, 1e-3, 1e-2):
            rhi, ylo, yhi = rlo + width, 0.001, 0.003
            got = O.payoff_cell(p, rlo, rhi, ylo, yhi)
            ym, hy, S = (mp.mpf(ylo) + mp.mpf(yhi)) / 2, (mp.mpf(yhi) - mp.mpf(ylo)) / 2, mp.mpf(0)
            for xk, wk in zip(xq, wq):
                cy = cm * mp.exp(-Gm * Gm * (ym + hy * mp.mpf(xk)) / 2)
                rs = mp.log(cy) / Gm
                a, b, sg = mp.mpf(rlo), mp.mpf(rhi), 1
                if kind == W.CAPLET:
                    a = max(a, rs)
                elif kind == W.FLOORLET:
                    b, sg = min(b, rs), -1
                if b > a:
                    S += mp.mpf(wk) * sg * ((b - a) - cy * (mp.exp(-Gm * a) - mp.exp(-Gm * b)) / Gm)
            want = float(S / 2 / (mp.mpf(rhi) - mp.mpf(rlo)))
            worst = max(worst, abs(got - want))
    assert worst <= 8 * np.finfo(float).eps, worst
