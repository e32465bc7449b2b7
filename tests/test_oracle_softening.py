"""Pins of the oracle's softened terminal data (section 7.2: the payoff
averaged over each node's control element).

F1: the Gauss-Legendre rule equals numpy's (leggauss) and integrates
polynomials up to degree 2n - 1 exactly.
F2: each cell average equals a brute-force double integral of the pointwise
payoff (scipy dblquad) over the same rectangle, on cells across the kink,
in the money and out of the money, for caplet, floorlet, forward and bond,
within the y rule's error (5e-9 relative).
F3: the averaged terminal grid keeps the pointwise data on Dirichlet nodes,
and the averages over a partition of a rectangle add up to the integral
over it.
"""
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


def test_terminal_grid_softened():
    s = W.with_shape(W.config1()[1], 24, 6, 12, 10)
    p = to_oracle(s)
    U0 = O.terminal(p)
    p.soften = 1
    U1 = O.terminal(p)
    r, _, _ = O.axis(p.axes[0])
    y, _, _ = O.axis(p.axes[2])
    # Dirichlet nodes (r_max, y_max) keep the pointwise payoff; v does not matter
    assert np.array_equal(U1[:, :, -1], U0[:, :, -1]) and np.array_equal(U1[-1], U0[-1])
    assert np.all(U1 == U1[:, :1, :])
    # the averages differ from the pointwise data near the kink only
    d = np.abs(U1 - U0)[0, 0, :-1]
    assert d.max() > 1e-5
    # cells partition [r_0, r_mid] x [y_0, y_mid] away from the Dirichlet faces:
    # sum of area x average = the integral over the union
    ih, kh = 10, 6
    rb = np.concatenate([[r[0]], 0.5 * (r[:-1] + r[1:])])
    yb = np.concatenate([[y[0]], 0.5 * (y[:-1] + y[1:])])
    total = sum((rb[i + 1] - rb[i]) * (yb[k + 1] - yb[k]) * U1[k, 0, i] for i in range(ih) for k in range(kh))
    want, _ = integrate.dblquad(lambda yy, rr: O.payoff(p, rr, yy), rb[0], rb[ih], yb[0], yb[kh],
                                epsabs=1e-15, epsrel=1e-12)
    assert abs(total - want) <= 5e-9 * abs(want), (total, want)
