"""Seeded synthetic workloads.

This module holds input recipes only: parameter sets, seeded draws and the
mesh layout of each workload.  It contains none of the pricing method's
arithmetic and imports nothing from the rest of the package, so both the GPU
path and the CPU oracle can be fed from it.

Parameter values follow the paper's "2007 market" set (section 3.3:
lambda = 0.15, gamma = 0.9, theta = 0.25) and its metric choice (section 7.1,
scaled units r0 = 0.01: r and y up to 250, v up to 30, stretch 0.5), converted
to physical units:  r in [0, 2.5] with alpha_r = 0.005 centred on the strike,
v in [0, 30] with alpha_v = 0.5 centred on 0.5, y in [0, 0.025] with
alpha_y = 5e-5 centred on 0.  The paper's figures and its discrete market
curve are not available, so every curve is the parametric
f(0,t) = level + slope (1 - exp(-decay t)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List, Optional, Tuple

import numpy as np

OUTFLOW = 0
DIRICHLET = 1
BOND, CAPLET, FLOORLET, FORWARD = 0, 1, 2, 3
# ADI schemes: the paper's Douglas, Craig-Sneyd, modified Craig-Sneyd,
# Hundsdorfer-Verwer (usual theta: 1/2, 1/2, 1/3, 1/2 + sqrt(3)/6), and
# Douglas with Huang's approximate-factorisation correction (af_iters
# subiterations)
DOUGLAS, CS, MCS, HV, HUANG = 0, 1, 2, 3, 4

LAMBDA = 0.15
GAMMA = 0.9
THETA_V = 0.25

R_MAX, ALPHA_R = 2.5, 0.005
V_MAX, ALPHA_V, CENTER_V = 30.0, 0.5, 0.5
Y_MAX, ALPHA_Y = 0.025, 5e-5


@dataclass(frozen=True)
class AxisSpec:
    n: int
    z_min: float
    z_max: float
    center: float
    alpha: float
    lo_face: int = OUTFLOW
    hi_face: int = OUTFLOW


@dataclass(frozen=True)
class ModelSpec:
    kappa: float
    epsilon: float
    rho: float
    f_level: float
    f_slope: float = 0.0
    f_decay: float = 0.0
    theta_v: float = THETA_V
    lam: float = LAMBDA
    gamma: float = GAMMA
    # a discrete initial curve (section 6.1) replaces the parametric one when
    # given: maturities (from 0) and zero-coupon prices (from 1)
    curve_t: Optional[Tuple[float, ...]] = None
    curve_p: Optional[Tuple[float, ...]] = None


@dataclass(frozen=True)
class PayoffSpec:
    kind: int
    expiry: float
    pay: float
    strike: float
    soften: int = 0   # 1: terminal data averaged over control elements (section 7.2)


@dataclass(frozen=True)
class SolveSpec:
    axes: Tuple[AxisSpec, AxisSpec, AxisSpec]
    model: ModelSpec
    payoff: PayoffSpec
    n_steps: int
    r0: float
    v0: float = 1.0
    scheme: int = 0      # ADI scheme: DOUGLAS (the paper's), CS, MCS, HV or HUANG
    theta: float = 0.5   # implicit weight of the line solves
    af_iters: int = 0    # HUANG: correction subiterations after the Douglas increment

    @property
    def shape(self):
        return (self.axes[2].n, self.axes[1].n, self.axes[0].n)

    @property
    def points(self) -> int:
        return self.axes[0].n * self.axes[1].n * self.axes[2].n


def default_axes(nr: int, nv: int, ny: int, center_r: float,
                 r_min: float = 0.0, r_lo_face: int = OUTFLOW) -> Tuple[AxisSpec, AxisSpec, AxisSpec]:
    """Default mesh: outflow at r = 0, v = 0, v = v_max, y = 0; Dirichlet at r_max, y_max."""
    return (AxisSpec(nr, r_min, R_MAX, center_r, ALPHA_R, r_lo_face, DIRICHLET),
            AxisSpec(nv, 0.0, V_MAX, CENTER_V, ALPHA_V, OUTFLOW, OUTFLOW),
            AxisSpec(ny, 0.0, Y_MAX, 0.0, ALPHA_Y, OUTFLOW, DIRICHLET))


def curve_integral(m: ModelSpec, t: float) -> float:
    """int_0^t f(0,s) ds for the parametric curve (input recipe for strikes)."""
    if m.f_decay == 0.0:
        return m.f_level * t
    return m.f_level * t + m.f_slope * (t - (1.0 - math.exp(-m.f_decay * t)) / m.f_decay)


def atm_strike(m: ModelSpec, expiry: float, pay: float) -> float:
    """Simple-compounded forward rate over [expiry, pay]: the at-the-money strike."""
    ratio = math.exp(curve_integral(m, pay) - curve_integral(m, expiry))
    return (ratio - 1.0) / (pay - expiry)


CURVE_SLOPED = dict(f_level=0.02, f_slope=0.01, f_decay=0.5)

# Maturities (years) of the synthetic discrete zero-coupon curve that stands
# in for the paper's market curve (figure 5, not available).
CURVE_KNOTS = (0.0, 0.25, 0.5, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 10.0, 12.0, 15.0, 20.0)


def discrete_curve(seed: int, knots: Tuple[float, ...] = CURVE_KNOTS) -> Tuple[Tuple[float, ...], Tuple[float, ...]]:
    """Seeded discrete zero-coupon curve: zero rates z(t) = a + b (1 - e^{-t/3})
    + h (t/2) e^{1 - t/2} with a ~ U[0.015, 0.03], b ~ U[0.005, 0.02] and a
    hump h ~ U[0, 0.004] near 2 y; prices P = e^{-z t} quoted to 5 decimals
    (the rounding makes the data discrete-valued, as market quotes are), and
    P(0, 0) = 1.  Returns (maturities, prices)."""
    rng = np.random.default_rng(seed)
    a, b, h = rng.uniform(0.015, 0.03), rng.uniform(0.005, 0.02), rng.uniform(0.0, 0.004)
    t = np.asarray(knots, dtype=np.float64)
    z = a + b * (1.0 - np.exp(-t / 3.0)) + h * (t / 2.0) * np.exp(1.0 - t / 2.0)
    P = np.round(np.exp(-z * t), 5)
    P[0] = 1.0
    return tuple(float(x) for x in t), tuple(float(x) for x in P)


def knot_atm_strike(curve_t, curve_p, expiry: float, pay: float) -> float:
    """The simple-compounded forward between two knots of a discrete curve."""
    i, j = curve_t.index(expiry), curve_t.index(pay)
    return (curve_p[i] / curve_p[j] - 1.0) / (pay - expiry)


def _draw_model(rng: np.random.Generator, **curve) -> ModelSpec:
    kappa = float(rng.uniform(0.01, 0.2))
    eps = float(rng.uniform(0.1, 0.6))
    rho = float(rng.uniform(-0.8, 0.8))
    return ModelSpec(kappa=kappa, epsilon=eps, rho=rho, **curve)


def config1() -> List[SolveSpec]:
    """32^3, 50 steps to T = 1y, flat 3 %, kappa 0.05, eps 0.3, rho -0.5: bond and ATM caplet."""
    m = ModelSpec(kappa=0.05, epsilon=0.3, rho=-0.5, f_level=0.03)
    k = atm_strike(m, 1.0, 2.0)
    bond = SolveSpec(default_axes(32, 32, 32, 0.03), m, PayoffSpec(BOND, 1.0, 2.0, k), 50, m.f_level)
    cap = SolveSpec(default_axes(32, 32, 32, k), m, PayoffSpec(CAPLET, 1.0, 2.0, k), 50, m.f_level)
    return [bond, cap]


def config2() -> List[SolveSpec]:
    """128x64x64, 200 steps to 5y, sloped curve, seed 1; caplets at ATM-100bp, ATM, ATM+100bp."""
    rng = np.random.default_rng(1)
    m = _draw_model(rng, **CURVE_SLOPED)
    k = atm_strike(m, 5.0, 6.0)
    ax = default_axes(128, 64, 64, k)
    return [SolveSpec(ax, m, PayoffSpec(CAPLET, 5.0, 6.0, k + dk), 200, m.f_level)
            for dk in (-0.01, 0.0, 0.01)]


def config3() -> List[SolveSpec]:
    """256x128x128, dt = 0.025 (400 steps to 10y), seed 2; ATM caplets expiring 1..10y, paid +1y."""
    rng = np.random.default_rng(2)
    m = _draw_model(rng, **CURVE_SLOPED)
    out = []
    for T in range(1, 11):
        k = atm_strike(m, float(T), float(T + 1))
        out.append(SolveSpec(default_axes(256, 128, 128, k), m,
                             PayoffSpec(CAPLET, float(T), float(T + 1), k), 40 * T, m.f_level))
    return out


def config_discrete(n: Tuple[int, int, int] = (128, 64, 64), seed: int = 4) -> List[SolveSpec]:
    """Caplets on the seeded discrete curve (section 6.1's second example):
    ATM, expiring 1, 2 and 5 y, paid +1 y, 40 steps a year, on a 128x64x64
    mesh; kappa ~ U[0.05, 0.2] (the r = 0 outflow face needs
    f_t + kappa f > 0, and the spline's f_t dips below 0 where the curve
    flattens), epsilon, rho as in the other configs.  r0 = the first knot
    interval's average rate."""
    rng = np.random.default_rng(seed)
    ct, cp = discrete_curve(seed)
    m = ModelSpec(kappa=float(rng.uniform(0.05, 0.2)), epsilon=float(rng.uniform(0.1, 0.6)),
                  rho=float(rng.uniform(-0.8, 0.8)), f_level=0.0, curve_t=ct, curve_p=cp)
    r0 = -math.log(cp[1]) / ct[1]
    out = []
    for T in (1.0, 2.0, 5.0):
        k = knot_atm_strike(ct, cp, T, T + 1.0)
        out.append(SolveSpec(default_axes(*n, k), m, PayoffSpec(CAPLET, T, T + 1.0, k), int(40 * T), r0))
    return out


def config4(n: int = 512, seed: int = 3) -> List[SolveSpec]:
    """Batched calibration-style solves: per solve n_r, n_v, n_y ~ U{32,48,64,96}, N ~ U{50..200},
    expiry ~ U{1..5}y paid +1y, strike ATM + U{-100,0,+100} bp, parameters as config 2."""
    rng = np.random.default_rng(seed)
    sizes = (32, 48, 64, 96)
    out = []
    for _ in range(n):
        nr, nv, ny = (int(sizes[rng.integers(0, 4)]) for _ in range(3))
        N = int(rng.integers(50, 201))
        m = _draw_model(rng, **CURVE_SLOPED)
        T = float(rng.integers(1, 6))
        dk = float((-0.01, 0.0, 0.01)[rng.integers(0, 3)])
        k = atm_strike(m, T, T + 1.0) + dk
        out.append(SolveSpec(default_axes(nr, nv, ny, k), m, PayoffSpec(CAPLET, T, T + 1.0, k), N, m.f_level))
    return out


# Surrogate box (8 inputs): kappa, eps, rho, v0, curve level, curve slope, strike offset, expiry.
SURROGATE_BOX_LO = np.array([0.01, 0.1, -0.8, 0.5, 0.01, 0.0, -0.01, 0.5])
SURROGATE_BOX_HI = np.array([0.2, 0.6, 0.8, 1.5, 0.04, 0.02, 0.01, 5.0])
SURROGATE_DT = 0.025
SURROGATE_N = 64
SURROGATE_F_DECAY = 0.5   # f(0,t) = level + slope (1 - exp(-SURROGATE_F_DECAY t))
SURROGATE_TENOR = 1.0     # the caplet pays one tenor after expiry
SURROGATE_V0 = tuple(0.5 + (1.5 - 0.5) * (q + 0.5) / 16.0 for q in range(16))


def surrogate_solve(x: np.ndarray, n: int = SURROGATE_N, soften: int = 0) -> SolveSpec:
    """One caplet solve from a surrogate input row (v0 is read out, not solved for);
    soften selects the terminal data (0 pointwise, 1 or 2 control-element averages)."""
    kappa, eps, rho, v0, lvl, slope, dk, T = (float(t) for t in x)
    m = ModelSpec(kappa=kappa, epsilon=eps, rho=rho, f_level=lvl, f_slope=slope, f_decay=SURROGATE_F_DECAY)
    k = atm_strike(m, T, T + SURROGATE_TENOR) + dk
    N = max(1, int(round(T / SURROGATE_DT)))
    return SolveSpec(default_axes(n, n, n, k), m, PayoffSpec(CAPLET, T, T + SURROGATE_TENOR, k, soften), N, lvl, v0)


def surrogate_readouts(n_solves: int, readouts: int, seed: int) -> np.ndarray:
    """v0 values (n_solves, readouts) at which each training solve is read out:
    the 16-point grid SURROGATE_V0 for every solve when readouts = 16, else
    seeded uniform draws in the box's v0 range."""
    if readouts == len(SURROGATE_V0):
        return np.tile(np.array(SURROGATE_V0), (n_solves, 1))
    rng = np.random.default_rng(seed)
    return SURROGATE_BOX_LO[3] + (SURROGATE_BOX_HI[3] - SURROGATE_BOX_LO[3]) * rng.random((n_solves, readouts))


def surrogate_params(n_solves: int, seed: int) -> np.ndarray:
    """Uniform draws in the surrogate box, one row per solve (column 3, v0, is overwritten
    by the readout grid of SURROGATE_V0 when the training set is built)."""
    rng = np.random.default_rng(seed)
    return SURROGATE_BOX_LO + (SURROGATE_BOX_HI - SURROGATE_BOX_LO) * rng.random((n_solves, 8))


# Coordinates that can leave the box while the problem stays valid for the
# solver (|rho| <= 1, epsilon >= 0, a forward curve that keeps the r = 0 face
# outflowing, a positive strike): (column, side) with side -1 below the box,
# +1 above.
_OUTSIDE_MOVES = ((0, +1), (3, -1), (3, +1), (4, +1), (6, +1), (7, +1))


def surrogate_outside(n: int, seed: int) -> np.ndarray:
    """Rows with one coordinate pushed 5-30 % of its span outside the box
    (fallback routing test); only moves that keep the problem valid."""
    rng = np.random.default_rng(seed)
    x = surrogate_params(n, seed + 1000)
    span = SURROGATE_BOX_HI - SURROGATE_BOX_LO
    for r in range(n):
        c, side = _OUTSIDE_MOVES[int(rng.integers(0, len(_OUTSIDE_MOVES)))]
        d = span[c] * float(rng.uniform(0.05, 0.3))
        x[r, c] = SURROGATE_BOX_LO[c] - d if side < 0 else SURROGATE_BOX_HI[c] + d
    return x


def gaussian_variant(s: SolveSpec, lam: float = 0.01, r_min: float = -0.5) -> SolveSpec:
    """Deterministic-volatility limit: gamma = 0, epsilon = 0, v0 = 1, negative rates allowed
    (both r faces Dirichlet)."""
    m = replace(s.model, gamma=0.0, epsilon=0.0, lam=lam)
    ax = default_axes(s.axes[0].n, s.axes[1].n, s.axes[2].n, s.axes[0].center,
                      r_min=r_min, r_lo_face=DIRICHLET)
    return replace(s, axes=ax, model=m, v0=1.0)


def with_shape(s: SolveSpec, nr: int, nv: int, ny: int, n_steps: int | None = None) -> SolveSpec:
    """Same problem on another mesh (and optionally another step count)."""
    ax = tuple(replace(a, n=n) for a, n in zip(s.axes, (nr, nv, ny)))
    return replace(s, axes=ax, n_steps=s.n_steps if n_steps is None else n_steps)


def spec_line(s: SolveSpec) -> str:
    """One solve as the 37 numbers the hjm_run command-line runner reads:
    3 x (n z_min z_max center alpha lo_face hi_face), the model, the payoff,
    then n_steps r0 v0."""
    if s.model.curve_t is not None:
        raise ValueError("the runner's spec lines carry the parametric curve only")
    f = []
    for a in s.axes:
        f += [a.n, a.z_min, a.z_max, a.center, a.alpha, a.lo_face, a.hi_face]
    m = s.model
    f += [m.kappa, m.theta_v, m.lam, m.gamma, m.epsilon, m.rho, m.f_level, m.f_slope, m.f_decay]
    f += [s.payoff.kind, s.payoff.expiry, s.payoff.pay, s.payoff.strike, s.n_steps, s.r0, s.v0]
    return " ".join(repr(float(x)) if isinstance(x, float) else str(int(x)) for x in f)


WORKLOADS = {"config1": config1, "config2": config2, "config3": config3, "config4": config4}


if __name__ == "__main__":
    import sys
    names = sys.argv[1:] or ["config3"]
    for name in names:
        if name not in WORKLOADS:
            sys.exit(f"unknown workload {name!r}; one of {sorted(WORKLOADS)}")
        print(f"# {name}: {WORKLOADS[name].__doc__.splitlines()[0]}")
        for s in WORKLOADS[name]():
            print(spec_line(s))
