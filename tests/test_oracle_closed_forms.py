"""Pins of the oracle's curve, bond formula, payoffs and Gaussian caplet closed form.

Each check compares the oracle with something the paper or mathematics fixes
independently of the oracle's own formula: integrals and derivatives of the
curve (section 2), the PDE of section 3.2 (eq. (1)) satisfied by the bond
formula eq. (gs), and the caplet of the Gaussian limit priced by direct
numerical integration over the lognormal bond price.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W


def sloped():
    return to_oracle(W.config2()[1])


def flat():
    return to_oracle(W.config1()[1])


@pytest.mark.parametrize("mk", [sloped, flat])
def test_discount_is_exp_of_minus_integrated_forward(mk):
    p = mk()
    for t in [0.0, 0.3, 1.0, 4.7, 10.0]:
        integral, _ = integrate.quad(lambda s: O.forward(p, s), 0.0, t, epsabs=1e-15, epsrel=1e-14)
        assert O.discount(p, t) == pytest.approx(math.exp(-integral), rel=1e-13, abs=1e-15)


def test_forward_slope_is_derivative_of_forward():
    p = sloped()
    h = 1e-5
    for t in [0.0, 0.5, 2.0, 9.0]:
        fd = (O.forward(p, t + h) - O.forward(p, t - h)) / (2 * h)
        assert O.forward_dt(p, t) == pytest.approx(fd, rel=1e-8)
    assert O.forward_dt(flat(), 3.0) == 0.0


def test_G_definition():
    # G(0) = 0, G'(s) = exp(-kappa s), G -> s as kappa -> 0
    assert O.G(0.05, 0.0) == 0.0
    h = 1e-5
    for kap in [0.001, 0.05, 0.2]:
        for s in [0.0, 1.0, 7.5]:
            d = (O.G(kap, s + h) - O.G(kap, s - h)) / (2 * h)
            assert d == pytest.approx(math.exp(-kap * s), rel=1e-8)
    assert O.G(0.0, 3.0) == 3.0
    assert O.G(1e-12, 3.0) == pytest.approx(3.0, rel=1e-10)


def test_bond_boundary_values():
    p = sloped()
    T = 5.0
    # p(T,T) = 1 at any state
    for r, y in [(0.0, 0.0), (0.05, 1e-4), (2.5, 0.02)]:
        assert O.bond(p, T, T, r, y) == pytest.approx(1.0, abs=1e-15)
    # x = r - f(0,t) = 0 and y = 0 give the forward discount factor
    for t in [0.0, 1.0, 3.0]:
        r = O.forward(p, t)
        assert O.bond(p, t, T, r, 0.0) == pytest.approx(O.discount(p, T) / O.discount(p, t), rel=1e-14)


def _pde_residual(p, t, r, v, y, T):
    """Residual of eq. (1) for C(t,r,y) = bond price; coefficients as printed in
    section 3.2 with the exponent of r read as gamma.  Finite differences."""
    C = lambda tt, rr, yy: O.bond(p, tt, T, rr, yy)
    ht, hr, hy = 1e-4, 1e-4, 1e-6
    Ct = (C(t + ht, r, y) - C(t - ht, r, y)) / (2 * ht)
    Cr = (C(t, r + hr, y) - C(t, r - hr, y)) / (2 * hr)
    Crr = (C(t, r + hr, y) - 2 * C(t, r, y) + C(t, r - hr, y)) / hr ** 2
    Cy = (C(t, r, y + hy) - C(t, r, y - hy)) / (2 * hy)
    lam, gam, kap = p.lam, p.gamma, p.kappa
    zeta_rr = 0.5 * lam ** 2 * r ** (2 * gam) * v
    mu_r = O.forward_dt(p, t) - kap * (r - O.forward(p, t)) + y
    mu_y = lam ** 2 * r ** (2 * gam) * v - 2 * kap * y
    # C does not depend on v, so the v and mixed terms vanish
    return Ct + zeta_rr * Crr + mu_r * Cr + mu_y * Cy - r * C(t, r, y), r * C(t, r, y)


@pytest.mark.parametrize("mk", [sloped, flat])
def test_bond_formula_solves_the_pricing_pde(mk):
    p = mk()
    rng = np.random.default_rng(11)
    for _ in range(20):
        t = rng.uniform(0.0, 4.0)
        r = rng.uniform(0.005, 0.3)
        v = rng.uniform(0.2, 3.0)
        y = rng.uniform(1e-5, 5e-3)
        res, scale = _pde_residual(p, t, r, v, y, 5.0)
        assert abs(res) < 2e-6 * max(scale, 1e-3), (t, r, v, y, res)


def test_bond_formula_fails_pde_when_a_term_is_dropped():
    # sanity of the residual check itself: dropping the -1/2 G^2 y term breaks it
    p = sloped()
    t, r, v, y, T = 1.0, 0.04, 1.0, 2e-3, 5.0
    G = O.G(p.kappa, T - t)
    wrong = O.bond(p, t, T, r, y) * math.exp(0.5 * G * G * y)
    ok = O.bond(p, t, T, r, y)
    assert abs(wrong - ok) > 1e-4 * ok


def test_payoffs_and_dirichlet_data():
    p = flat()
    T, TM, K = p.expiry, p.pay, p.strike
    D = 1.0 + (TM - T) * K
    for r, y in [(0.0, 0.0), (0.03, 0.0), (0.1, 1e-3), (2.5, 0.025)]:
        pm = O.bond(p, T, TM, r, y)
        p.kind = W.CAPLET
        cap = O.payoff(p, r, y)
        assert cap == pytest.approx(max(1 - D * pm, 0.0), abs=1e-16)
        p.kind = W.FLOORLET
        flo = O.payoff(p, r, y)
        p.kind = W.FORWARD
        lin = O.payoff(p, r, y)
        assert cap - flo == lin  # max(x,0) - max(-x,0) = x exactly
        p.kind = W.BOND
        assert O.payoff(p, r, y) == 1.0
        # Dirichlet data at t = T coincide with the payoff
        for kind in (W.BOND, W.CAPLET, W.FLOORLET, W.FORWARD):
            p.kind = kind
            assert O.dirichlet(p, T, r, y) == pytest.approx(O.payoff(p, r, y), abs=1e-15)
    p.kind = W.CAPLET


@pytest.mark.parametrize("kappa,lam,T,dk", [(0.05, 0.01, 1.0, 0.0), (0.15, 0.008, 5.0, 0.01),
                                             (0.01, 0.012, 3.0, -0.01), (0.0, 0.01, 2.0, 0.005)])
def test_gaussian_caplet_against_numerical_integration(kappa, lam, T, dk):
    """Gaussian limit (gamma = 0, eps = 0, v = 1): ln p(T,T_M) is normal under the
    T-forward measure with mean ln(P_M/P_T) - s^2/2, variance s^2 = G^2 Var x(T),
    Var x(T) = int_0^T lam^2 exp(-2 kappa (T-u)) du.  Integrate the payoff."""
    base = W.config2()[1]
    m = W.ModelSpec(kappa=kappa, epsilon=0.0, rho=0.0, f_level=0.02, f_slope=0.01, f_decay=0.5,
                    lam=lam, gamma=0.0)
    K = W.atm_strike(m, T, T + 1.0) + dk
    s = W.SolveSpec(base.axes, m, W.PayoffSpec(W.CAPLET, T, T + 1.0, K), 10, 0.02)
    p = to_oracle(s)
    var_x, _ = integrate.quad(lambda u: lam ** 2 * math.exp(-2 * kappa * (T - u)), 0.0, T, epsabs=1e-16)
    Gm = (T + 1.0 - T) if kappa == 0 else (1 - math.exp(-kappa * 1.0)) / kappa
    sd = Gm * math.sqrt(var_x)
    PT, PM = O.discount(p, T), O.discount(p, T + 1.0)
    D = 1 + K
    mean = math.log(PM / PT) - 0.5 * sd * sd
    dens = lambda z: math.exp(-0.5 * ((z - mean) / sd) ** 2) / (sd * math.sqrt(2 * math.pi))
    kink = -math.log(D)
    val, _ = integrate.quad(lambda z: (1 - D * math.exp(z)) * dens(z), mean - 12 * sd, kink,
                            epsabs=1e-15, epsrel=1e-12, limit=200)
    assert O.gaussian_caplet(p) == pytest.approx(PT * val, rel=1e-9)
