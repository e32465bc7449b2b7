"""Pins of the oracle's Greeks readout (rho = dC/dr, vega = dC/dv at (r0, v0)
on the y_min plane, section 6).

G1: on a field that is a cubic polynomial in each mesh coordinate the 4-point
interpolant is exact, so its derivatives equal the chain rule P'(x_r) x_r'(r)
Q(x_v) (and the same in v), with x'(z) from differentiating the inverse map by
hand; a wrong basis derivative or a missing metric factor fails.
G2: the derivatives agree with central differences of the oracle's own
price readout, moved inside one mesh interval (brute force).
G3: the bond's exact price does not depend on v, so its discrete vega falls
with the mesh, and its rho approaches the closed form dp(0,T)/dr =
-G(T) p(0,T).
"""
import math

import numpy as np
import pytest

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W


def _dxdz(ax, z):
    c1 = math.asinh((ax.z_min - ax.center) / ax.alpha)
    c2 = math.asinh((ax.z_max - ax.center) / ax.alpha)
    return 1.0 / ((c2 - c1) * math.sqrt(ax.alpha ** 2 + (z - ax.center) ** 2))


def test_greeks_exact_on_cubic_fields():
    p = to_oracle(W.with_shape(W.config1()[1], 24, 20, 6, 10))
    nr, nv, ny = (a.n for a in p.axes)
    xr = np.linspace(0.0, 1.0, nr)
    xv = np.linspace(0.0, 1.0, nv)
    P = lambda x: 0.3 - 1.7 * x + 2.1 * x ** 2 - 0.9 * x ** 3
    dP = lambda x: -1.7 + 4.2 * x - 2.7 * x ** 2
    Q = lambda x: 1.2 + 0.5 * x - 3.0 * x ** 2 + 1.1 * x ** 3
    dQ = lambda x: 0.5 - 6.0 * x + 3.3 * x ** 2
    U = np.zeros((ny, nv, nr))
    U[:] = Q(xv)[None, :, None] * P(xr)[None, None, :]
    for r0, v0 in [(0.031, 1.0), (0.0007, 0.3), (0.9, 7.5), (2.2, 25.0)]:
        ar, av = p.axes[0], p.axes[1]
        x_r = O.axis_x(ar, r0)
        x_v = O.axis_x(av, v0)
        want = [P(x_r) * Q(x_v), dP(x_r) * _dxdz(ar, r0) * Q(x_v), P(x_r) * dQ(x_v) * _dxdz(av, v0)]
        got = O.greeks(p, U, r0, v0)
        assert np.allclose(got, want, rtol=1e-11, atol=1e-11 * max(abs(x) for x in want)), (r0, v0, got, want)


def test_greeks_match_differences_of_the_readout():
    s = W.with_shape(W.config1()[1], 32, 24, 12, 20)
    p = to_oracle(s)
    _, U = O.price(p, s.r0, s.v0)
    g = O.greeks(p, U, s.r0, s.v0)
    assert g[0] == O.readout(p, U, s.r0, s.v0)
    hr, hv = 1e-6 * s.r0, 1e-6
    dr = (O.readout(p, U, s.r0 + hr, s.v0) - O.readout(p, U, s.r0 - hr, s.v0)) / (2 * hr)
    dv = (O.readout(p, U, s.r0, s.v0 + hv) - O.readout(p, U, s.r0, s.v0 - hv)) / (2 * hv)
    assert abs(g[1] - dr) <= 1e-6 * abs(dr)
    assert abs(g[2] - dv) <= 1e-5 * abs(dv) + 1e-12


def test_bond_vega_vanishes_and_rho_converges():
    """The bond formula solves the pricing PDE for every v (the v terms cancel
    between the r diffusion and the y drift), so the discrete vega is a
    discretisation error that falls with the mesh, and rho tends to
    -G(T) p(0,T)."""
    errs, vegas = [], []
    for n in (16, 32, 48):
        s = W.with_shape(W.config1()[0], n, n, n, 200)
        p = to_oracle(s)
        _, U = O.price(p, s.r0, s.v0)
        c, rho, vega = O.greeks(p, U, s.r0, s.v0)
        exact = -O.G(p.kappa, p.expiry) * O.discount(p, p.expiry)
        errs.append(abs(rho - exact) / abs(exact))
        vegas.append(abs(vega) / abs(exact))
    assert errs[-1] < 1e-3 and errs[0] > errs[-1], errs
    assert vegas[-1] < 1e-4 and vegas[0] > 2.0 * vegas[-1], vegas
