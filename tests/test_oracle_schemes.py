"""Pins of the oracle's correction schemes (Craig-Sneyd, modified Craig-Sneyd,
Hundsdorfer-Verwer) next to the paper's Douglas scheme.

S1: one step of each scheme satisfies its defining stage equations, checked
with dense matrices built from the oracle's operators (as P7 does for
Douglas): with M_d = I - theta dt A_d, D0 the explicit predictor and
D3 = (M_r M_v M_y)^{-1} D0 the Douglas increment, the step's increment solves
M_r M_v M_y E3 = E0 for the scheme's corrected start E0 (U^{n+1} - U^n = E3,
or D3 + E3 for HV).  A wrong coefficient, a dropped term or the wrong
sweep order fails it.

S2: without a mixed term (rho = 0, so A0 = 0) Craig-Sneyd is the Douglas
scheme, bit for bit; with theta = 1/2 modified Craig-Sneyd is Craig-Sneyd,
bit for bit.

S3: with the mixed term present, one step of each of the three schemes
differs from one step of unsplit Crank-Nicolson (dense solve) by O(dt^3),
second-order accuracy, where Douglas differs by O(dt^2).

Huang's approximate-factorisation correction (section 5.1):
H1: with q subiterations the step equals the dense recursion
X_1 = M^{-1} D0, X_{m+1} = X_m + M^{-1} (D0 - (I - theta dt A) X_m) (the
residual zero on Dirichlet nodes), U^{n+1} = U^n + X_{q+1}.
H2: the subiterations converge to the unsplit theta step (a dense solve of
(I - theta dt A) X = D0): the distance falls geometrically with q and
reaches rounding; at q = 0 it is the Douglas step's factorisation error.
H3: one subiteration at theta = 1/2 is the Hundsdorfer-Verwer step at
theta = 1/2 (to rounding).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1108_1688_amd import workloads as W
from test_oracle_operators import _dense_ops, _dirichlet_mask, _small_problem

THETA_MCS = 1.0 / 3.0
THETA_HV = 0.5 + math.sqrt(3.0) / 6.0


def _g(p, t):
    r, _, _ = O.axis(p.axes[0])
    y, _, _ = O.axis(p.axes[2])
    return np.array([[[O.dirichlet(p, t, r[i], y[k]) for i in range(len(r))]
                      for _ in range(p.axes[1].n)] for k in range(len(y))]).ravel()


@pytest.mark.parametrize("scheme,theta", [(O.CS, 0.5), (O.MCS, THETA_MCS), (O.HV, THETA_HV), (O.DOUGLAS, 0.3)],
                         ids=["CS", "MCS", "HV", "Douglas-theta"])
@pytest.mark.parametrize("kind", [W.CAPLET, W.BOND])
def test_scheme_step_stage_equations(scheme, theta, kind):
    p = _small_problem(6, 5, 5)
    p.kind, p.scheme, p.theta = kind, scheme, theta
    n = 5
    dt = p.expiry / p.n_steps
    t_now, t_next, t_half = p.expiry - n * dt, p.expiry - (n + 1) * dt, p.expiry - (n + 0.5) * dt
    rng = np.random.default_rng(11)
    U0 = O.terminal(p) + 0.01 * rng.standard_normal(p.shape)
    U1 = O.step(p, n, U0.copy())
    Ar, Av, Ay, Ax = _dense_ops(p, t_half)
    A = Ar + Av + Ay + Ax
    I = np.eye(A.shape[0])
    Mr, Mv, My = I - theta * dt * Ar, I - theta * dt * Av, I - theta * dt * Ay
    M = Mr @ Mv @ My
    mask = _dirichlet_mask(p)
    inc = _g(p, t_next) - _g(p, t_now)
    D0 = dt * A @ U0.ravel()
    D0[mask] = inc[mask]
    D3 = np.linalg.solve(M, D0)
    if scheme == O.DOUGLAS:
        E0, step = D0, U1.ravel() - U0.ravel()
    elif scheme == O.CS:
        E0 = D0 + 0.5 * dt * Ax @ D3
        E0[mask] = inc[mask]
        step = U1.ravel() - U0.ravel()
    elif scheme == O.MCS:
        E0 = D0 + theta * dt * Ax @ D3 + (0.5 - theta) * dt * A @ D3
        E0[mask] = inc[mask]
        step = U1.ravel() - U0.ravel()
    else:
        E0 = D0 + 0.5 * dt * A @ D3 - D3
        E0[mask] = 0.0
        step = U1.ravel() - U0.ravel() - D3
    lhs = M @ step
    scale = max(np.abs(E0).max(), np.abs(D0).max())
    assert np.abs(lhs - E0).max() <= 1e-12 * scale
    if scheme != O.DOUGLAS:
        # the correction is not negligible: the plain Douglas increment fails
        assert np.abs(M @ (U1.ravel() - U0.ravel()) - D0).max() > 1e3 * np.abs(lhs - E0).max()


def test_cs_is_douglas_without_mixed_term():
    p = _small_problem(9, 8, 7, rho=0.0)
    U_d = O.run(p, 0, 6)
    p.scheme = O.CS
    U_c = O.run(p, 0, 6)
    assert np.array_equal(U_c, U_d)


def test_mcs_at_half_is_cs():
    p = _small_problem(9, 8, 7, rho=-0.6)
    p.scheme, p.theta = O.CS, 0.5
    U_c = O.run(p, 0, 6)
    p.scheme = O.MCS
    U_m = O.run(p, 0, 6)
    assert np.array_equal(U_c, U_m)
    p.scheme = O.DOUGLAS
    assert not np.array_equal(O.run(p, 0, 6), U_c)


@pytest.mark.parametrize("scheme,theta,order", [(O.CS, 0.5, 3), (O.MCS, THETA_MCS, 3), (O.HV, THETA_HV, 3),
                                                (O.DOUGLAS, 0.5, 2)], ids=["CS", "MCS", "HV", "Douglas"])
def test_local_error_against_unsplit_cn(scheme, theta, order):
    """One step from the same data against unsplit Crank-Nicolson (dense
    solve, the same Dirichlet increments), with dt small against the
    operator's spectral radius so that the error expansion in dt holds for
    every mode: the difference falls like dt^3 for the correction schemes
    (second order) and like dt^2 for Douglas, whose explicit mixed term is
    first order.  Halving dt divides it by 8 or by 4."""
    p = _small_problem(6, 5, 5, rho=-0.8)
    p.kind, p.epsilon = W.CAPLET, 0.6
    rng = np.random.default_rng(1)
    U0 = O.terminal(p) + 0.01 * rng.standard_normal(p.shape)
    mask = _dirichlet_mask(p)
    Ar, Av, Ay, Ax = _dense_ops(p, 0.5 * p.expiry)
    radius = np.abs(np.linalg.eigvals(Ar + Av + Ay + Ax)).max()
    errs = []
    for f in (1, 2, 4):
        N = int(round(p.expiry * radius / 1e-2)) * f
        dt = p.expiry / N
        p.scheme, p.theta, p.n_steps = O.DOUGLAS, 0.5, N
        Ar, Av, Ay, Ax = _dense_ops(p, p.expiry - 0.5 * dt)
        A = Ar + Av + Ay + Ax
        rhs = dt * A @ U0.ravel()
        rhs[mask] = (_g(p, p.expiry - dt) - _g(p, p.expiry))[mask]
        ucn = U0.ravel() + np.linalg.solve(np.eye(A.shape[0]) - 0.5 * dt * A, rhs)
        p.scheme, p.theta = scheme, theta
        errs.append(np.abs(O.step(p, 0, U0.copy()).ravel() - ucn).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    want = 2.0 ** order
    assert all(abs(r / want - 1.0) < 0.1 for r in ratios), (errs, ratios)


def _huang_setup(theta=0.5, rho=-0.6):
    p = _small_problem(6, 5, 5, rho=rho)
    p.kind = W.CAPLET
    n = 3
    dt = p.expiry / p.n_steps
    t_now, t_next, t_half = p.expiry - n * dt, p.expiry - (n + 1) * dt, p.expiry - (n + 0.5) * dt
    rng = np.random.default_rng(5)
    U0 = O.terminal(p) + 0.01 * rng.standard_normal(p.shape)
    Ar, Av, Ay, Ax = _dense_ops(p, t_half)
    A = Ar + Av + Ay + Ax
    I = np.eye(A.shape[0])
    M = (I - theta * dt * Ar) @ (I - theta * dt * Av) @ (I - theta * dt * Ay)
    mask = _dirichlet_mask(p)
    D0 = dt * A @ U0.ravel()
    D0[mask] = (_g(p, t_next) - _g(p, t_now))[mask]
    return p, n, U0, A, I, M, mask, D0, dt


@pytest.mark.parametrize("theta", [0.5, 0.7])
@pytest.mark.parametrize("q", [1, 2, 5])
def test_huang_subiterations_dense_recursion(q, theta):
    p, n, U0, A, I, M, mask, D0, dt = _huang_setup(theta)
    X = np.linalg.solve(M, D0)
    for _ in range(q):
        R = D0 - (I - theta * dt * A) @ X
        R[mask] = 0.0
        X = X + np.linalg.solve(M, R)
    p.scheme, p.theta, p.af_iters = O.HUANG, theta, q
    U1 = O.step(p, n, U0.copy())
    assert np.abs((U1.ravel() - U0.ravel()) - X).max() <= 1e-12 * np.abs(X).max()


def test_huang_converges_to_unsplit_step():
    theta = 0.5
    p, n, U0, A, I, M, mask, D0, dt = _huang_setup(theta)
    # the unsplit step: (I - theta dt A) X = D0 off the Dirichlet nodes, X = D0 on them
    K = I - theta * dt * A
    K[mask] = I[mask]
    X = np.linalg.solve(K, D0)
    p.scheme, p.theta = O.DOUGLAS, theta
    dist = [np.abs(O.step(p, n, U0.copy()).ravel() - U0.ravel() - X).max()]
    p.scheme = O.HUANG
    for q in range(1, 41):
        p.af_iters = q
        dist.append(np.abs(O.step(p, n, U0.copy()).ravel() - U0.ravel() - X).max())
    scale = np.abs(X).max()
    assert dist[0] > 1e-6 * scale          # the factorisation error of one Douglas step
    assert all(b < a for a, b in zip(dist[:8], dist[1:9])), dist[:9]
    assert dist[40] <= 1e-13 * scale, (dist[40], scale)


def test_huang_one_subiteration_is_hv_at_half():
    p = _small_problem(9, 8, 7, rho=-0.6)
    p.scheme, p.theta = O.HV, 0.5
    U_hv = O.run(p, 0, 6)
    p.scheme, p.af_iters = O.HUANG, 1
    U_h = O.run(p, 0, 6)
    assert np.abs(U_h - U_hv).max() <= 1e-14 * np.abs(U_hv).max()
    p.af_iters = 2
    assert np.abs(O.run(p, 0, 6) - U_hv).max() > 1e-10 * np.abs(U_hv).max()
