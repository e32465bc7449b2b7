"""CPU oracle for the single-factor HJM stochastic-volatility PDE.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports,
links or calls anything here, and nothing here imports the product package.

The arithmetic lives in ``hjm_oracle.c`` (plain FP64 C, one function per step of
the paper's method, built with ``-O2 -ffp-contract=off``).  This module only
marshals arguments through ctypes and builds the library with gcc if needed.

Functions without an independent pin are marked "parity unpinned" in their
docstrings; every other entry point is checked by ``tests/test_oracle_*.py``
against closed forms, invariants or brute force.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hjm_oracle.c")
_LIB = os.path.join(_HERE, "libhjm_oracle.so")

OUTFLOW = 0
DIRICHLET = 1
BOND, CAPLET, FLOORLET, FORWARD = 0, 1, 2, 3
# ADI schemes: the paper's Douglas, Craig-Sneyd, modified Craig-Sneyd,
# Hundsdorfer-Verwer, and Douglas with Huang's approximate-factorisation
# correction subiterations
DOUGLAS, CS, MCS, HV, HUANG = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("face", C.c_int * 6),
        ("geom", (C.c_double * 4) * 3),
        ("kappa", C.c_double), ("theta_v", C.c_double), ("lam", C.c_double),
        ("gamma", C.c_double), ("epsilon", C.c_double), ("rho", C.c_double),
        ("f_level", C.c_double), ("f_slope", C.c_double), ("f_decay", C.c_double),
        ("kind", C.c_int), ("expiry", C.c_double), ("pay", C.c_double),
        ("strike", C.c_double), ("n_steps", C.c_int),
        ("scheme", C.c_int), ("theta", C.c_double), ("soften", C.c_int), ("af_iters", C.c_int),
        ("curve_n", C.c_int), ("curve_t", C.POINTER(C.c_double)), ("curve_p", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        l = C.CDLL(build())
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        d = C.c_double
        sig = {
            "orc_set_threads": (None, [C.c_int]),
            "orc_get_threads": (C.c_int, []),
            "orc_forward": (d, [P, d]),
            "orc_forward_dt": (d, [P, d]),
            "orc_discount": (d, [P, d]),
            "orc_G": (d, [d, d]),
            "orc_bond": (d, [P, d, d, d, d]),
            "orc_payoff": (d, [P, d, d]),
            "orc_dirichlet": (d, [P, d, d, d]),
            "orc_gaussian_caplet": (d, [P]),
            "orc_axis": (None, [C.c_int, d, d, d, d, dp, dp, dp]),
            "orc_axis_x": (d, [d, d, d, d, d]),
            "orc_apply": (C.c_int, [P, C.c_int, d, dp, dp]),
            "orc_line_solve": (C.c_int, [C.c_int, dp, dp, dp, d, d, dp, dp]),
            "orc_step": (C.c_int, [P, C.c_int, dp]),
            "orc_terminal": (C.c_int, [P, dp]),
            "orc_run": (C.c_int, [P, C.c_int, C.c_int, dp]),
            "orc_bond_grid": (C.c_int, [P, d, dp]),
            "orc_readout": (d, [P, dp, d, d]),
            "orc_greeks": (None, [P, dp, d, d, dp]),
            "orc_gauss_legendre": (None, [C.c_int, dp, dp]),
            "orc_payoff_cell": (d, [P, d, d, d, d]),
            "orc_price": (C.c_int, [P, d, d, dp, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Axis:
    """One mesh axis: n nodes (both ends included) of the sinh map of section 4.3."""
    n: int
    z_min: float
    z_max: float
    center: float
    alpha: float
    lo_face: int = OUTFLOW
    hi_face: int = OUTFLOW


@dataclass
class Problem:
    """Everything that defines one discrete solve (oracle's own description)."""
    axes: Sequence[Axis]
    kappa: float
    theta_v: float
    lam: float
    gamma: float
    epsilon: float
    rho: float
    f_level: float
    f_slope: float = 0.0
    f_decay: float = 0.0
    kind: int = CAPLET
    expiry: float = 1.0
    pay: float = 2.0
    strike: float = 0.03
    n_steps: int = 50
    scheme: int = DOUGLAS
    theta: float = 0.5
    soften: int = 0
    af_iters: int = 0
    curve_t: Optional[Sequence[float]] = None   # discrete curve (section 6.1): maturities from 0
    curve_p: Optional[Sequence[float]] = None   # and zero-coupon prices from 1
    _c: _Problem = field(default=None, repr=False, compare=False)
    _knots: tuple = field(default=None, repr=False, compare=False)

    @property
    def shape(self):
        """Array shape of the grid, (ny, nv, nr): r is the fastest index."""
        return (self.axes[2].n, self.axes[1].n, self.axes[0].n)

    def c(self) -> _Problem:
        p = _Problem()
        for a in range(3):
            ax = self.axes[a]
            p.n[a] = ax.n
            p.face[2 * a] = ax.lo_face
            p.face[2 * a + 1] = ax.hi_face
            p.geom[a][0] = ax.z_min
            p.geom[a][1] = ax.z_max
            p.geom[a][2] = ax.center
            p.geom[a][3] = ax.alpha
        p.kappa, p.theta_v, p.lam = self.kappa, self.theta_v, self.lam
        p.gamma, p.epsilon, p.rho = self.gamma, self.epsilon, self.rho
        p.f_level, p.f_slope, p.f_decay = self.f_level, self.f_slope, self.f_decay
        p.kind, p.expiry, p.pay, p.strike = self.kind, self.expiry, self.pay, self.strike
        p.n_steps = self.n_steps
        p.scheme, p.theta = self.scheme, self.theta
        p.soften = self.soften
        p.af_iters = self.af_iters
        if self.curve_t is not None:
            t = np.ascontiguousarray(self.curve_t, dtype=np.float64)
            q = np.ascontiguousarray(self.curve_p, dtype=np.float64)
            if not (2 <= len(t) <= 64 and len(q) == len(t) and t[0] == 0.0 and q[0] == 1.0
                    and np.all(np.diff(t) > 0) and np.all(q > 0)):
                raise ValueError("discrete curve: 2..64 knots from (0, 1), increasing maturities, prices > 0")
            self._knots = (t, q)  # alive as long as the struct that points at them
            p.curve_n = len(t)
            p.curve_t = t.ctypes.data_as(C.POINTER(C.c_double))
            p.curve_p = q.ctypes.data_as(C.POINTER(C.c_double))
        self._c = p
        return p

    def ref(self):
        return C.byref(self.c())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def forward(p: Problem, t: float) -> float:
    return lib().orc_forward(p.ref(), t)


def forward_dt(p: Problem, t: float) -> float:
    return lib().orc_forward_dt(p.ref(), t)


def discount(p: Problem, t: float) -> float:
    return lib().orc_discount(p.ref(), t)


def G(kappa: float, s: float) -> float:
    return lib().orc_G(kappa, s)


def bond(p: Problem, t: float, T: float, r: float, y: float) -> float:
    return lib().orc_bond(p.ref(), t, T, r, y)


def payoff(p: Problem, r: float, y: float) -> float:
    return lib().orc_payoff(p.ref(), r, y)


def dirichlet(p: Problem, t: float, r: float, y: float) -> float:
    return lib().orc_dirichlet(p.ref(), t, r, y)


def gaussian_caplet(p: Problem) -> float:
    return lib().orc_gaussian_caplet(p.ref())


def axis(ax: Axis):
    z = np.empty(ax.n)
    J = np.empty(ax.n)
    J2 = np.empty(ax.n)
    lib().orc_axis(ax.n, ax.z_min, ax.z_max, ax.center, ax.alpha, _dp(z), _dp(J), _dp(J2))
    return z, J, J2


def axis_x(ax: Axis, z: float) -> float:
    return lib().orc_axis_x(z, ax.z_min, ax.z_max, ax.center, ax.alpha)


def apply(p: Problem, d: int, t: float, U: np.ndarray) -> np.ndarray:
    """A_d U at physical time t; d = 0 r, 1 v, 2 y, 3 mixed r-v."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty_like(U)
    rc = lib().orc_apply(p.ref(), d, t, _dp(U), _dp(out))
    if rc:
        raise RuntimeError(f"orc_apply failed: {rc}")
    return out


def line_solve(a, b, c, e_lo, e_hi, d) -> np.ndarray:
    a, b, c, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d))
    x = np.empty_like(d)
    rc = lib().orc_line_solve(len(d), _dp(a), _dp(b), _dp(c), e_lo, e_hi, _dp(d), _dp(x))
    if rc:
        raise RuntimeError(f"orc_line_solve failed: {rc}")
    return x


def terminal(p: Problem) -> np.ndarray:
    U = np.empty(p.shape)
    lib().orc_terminal(p.ref(), _dp(U))
    return U


def step(p: Problem, n: int, U: np.ndarray) -> np.ndarray:
    """One Douglas step tau_n -> tau_{n+1}, in place; returns U."""
    rc = lib().orc_step(p.ref(), n, _dp(U))
    if rc:
        raise RuntimeError(f"orc_step failed: {rc}")
    return U


def run(p: Problem, first: int = 0, last: int | None = None, U: np.ndarray | None = None) -> np.ndarray:
    """Terminal data (if first == 0) then steps [first, last)."""
    if last is None:
        last = p.n_steps
    if U is None:
        U = np.empty(p.shape)
    rc = lib().orc_run(p.ref(), first, last, _dp(U))
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    return U


def bond_grid(p: Problem, t: float) -> np.ndarray:
    out = np.empty(p.shape)
    lib().orc_bond_grid(p.ref(), t, _dp(out))
    return out


def readout(p: Problem, U: np.ndarray, r0: float, v0: float) -> float:
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_readout(p.ref(), _dp(U), r0, v0)


def gauss_legendre(n: int):
    x, w = np.empty(n), np.empty(n)
    lib().orc_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


def payoff_cell(p: Problem, rlo: float, rhi: float, ylo: float, yhi: float) -> float:
    """The terminal data averaged over [rlo, rhi] x [ylo, yhi] (section 7.2)."""
    return lib().orc_payoff_cell(p.ref(), rlo, rhi, ylo, yhi)


def greeks(p: Problem, U: np.ndarray, r0: float, v0: float) -> np.ndarray:
    """(C, dC/dr, dC/dv) at (r0, v0, y_min): the readout's interpolant and its
    derivatives (the rho and vega of section 6)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty(3)
    lib().orc_greeks(p.ref(), _dp(U), r0, v0, _dp(out))
    return out


def price(p: Problem, r0: float, v0: float = 1.0):
    """Full solve and readout; returns (price, final grid)."""
    U = np.empty(p.shape)
    out = C.c_double()
    rc = lib().orc_price(p.ref(), r0, v0, _dp(U), C.byref(out))
    if rc:
        raise RuntimeError(f"orc_price failed: {rc}")
    return out.value, U
