"""Pins of the oracle's discrete operators and Douglas step.

P8: on fields that are quadratic in each mesh coordinate the centred stencils
of eq. (esquema) (first difference over 2h, mixed over 4 h_r h_v) and the
one-sided outflow rows of section 7.3 are exact, so every directional operator
must equal the physical PDE terms of eq. (1) evaluated with the chain rule.
The derivatives of the mesh map used here come from differentiating the
inverse map x(z) = (asinh((z-K)/alpha) - c1)/(c2-c1) by hand, independently of
the oracle's Jacobian tables.

P7: the Douglas step of section 5.1 satisfies, with dense matrices built from
the oracle's own operators, M_r M_v M_y (U^{n+1} - U^n) = D0, where
M_d = I - theta dt A_d and D0 is the explicit predictor.

P9: with no mixed term the Douglas step differs from unsplit Crank-Nicolson
(dense solve) by a splitting error that is second order globally.
"""
import math

import numpy as np
import pytest

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W


def _inv_map_derivs(ax, z):
    c1 = math.asinh((ax.z_min - ax.center) / ax.alpha)
    c2 = math.asinh((ax.z_max - ax.center) / ax.alpha)
    q = ax.alpha ** 2 + (z - ax.center) ** 2
    d1 = 1.0 / ((c2 - c1) * np.sqrt(q))
    d2 = -(z - ax.center) / ((c2 - c1) * q ** 1.5)
    return d1, d2


def _small_problem(nr=9, nv=8, ny=7, rho=-0.5):
    s = W.config2()[1]
    m = W.ModelSpec(kappa=0.07, epsilon=0.4, rho=rho, **W.CURVE_SLOPED)
    s = W.SolveSpec(s.axes, m, s.payoff, 20, s.r0)
    return to_oracle(W.with_shape(s, nr, nv, ny))


def test_operators_exact_on_quadratic_fields():
    p = _small_problem()
    nr, nv, ny = (a.n for a in p.axes)
    rng = np.random.default_rng(5)
    cr, cv, cy = rng.standard_normal(3), rng.standard_normal(3), rng.standard_normal(3)
    P = lambda x: cr[0] + cr[1] * x + cr[2] * x * x
    Q = lambda x: cv[0] + cv[1] * x + cv[2] * x * x
    S = lambda x: cy[0] + cy[1] * x + cy[2] * x * x
    dP = lambda x: cr[1] + 2 * cr[2] * x
    dQ = lambda x: cv[1] + 2 * cv[2] * x
    dS = lambda x: cy[1] + 2 * cy[2] * x
    xr = np.arange(nr) / (nr - 1)
    xv = np.arange(nv) / (nv - 1)
    xy = np.arange(ny) / (ny - 1)
    U = S(xy)[:, None, None] * Q(xv)[None, :, None] * P(xr)[None, None, :]
    r, _, _ = O.axis(p.axes[0])
    v, _, _ = O.axis(p.axes[1])
    y, _, _ = O.axis(p.axes[2])
    r1, r2 = _inv_map_derivs(p.axes[0], r)
    v1, v2 = _inv_map_derivs(p.axes[1], v)
    y1, _ = _inv_map_derivs(p.axes[2], y)
    t = 2.3
    A = [O.apply(p, d, t, U) for d in range(4)]
    f, ft = O.forward(p, t), O.forward_dt(p, t)
    lam, gam, eps, kap = p.lam, p.gamma, p.epsilon, p.kappa
    checked = 0
    for k in range(ny):
        for j in range(nv):
            for i in range(nr):
                if i == nr - 1 or k == ny - 1:
                    assert all(a[k, j, i] == 0.0 for a in A)  # Dirichlet nodes
                    continue
                rr, vv, yy = r[i], v[j], y[k]
                # eq. (1) coefficients (exponent gamma)
                z_rr = 0.5 * lam ** 2 * rr ** (2 * gam) * vv
                z_vv = 0.5 * eps ** 2 * vv
                z_rv = lam * rr ** gam * eps * p.rho * vv
                mu_r = ft - kap * (rr - f) + yy
                mu_v = p.theta_v * (1 - vv)
                mu_y = lam ** 2 * rr ** (2 * gam) * vv - 2 * kap * yy
                Pi, Qj, Sk = P(xr[i]), Q(xv[j]), S(xy[k])
                Ur = dP(xr[i]) * r1[i] * Qj * Sk
                Urr = (2 * cr[2] * r1[i] ** 2 + dP(xr[i]) * r2[i]) * Qj * Sk
                Uv = Pi * dQ(xv[j]) * v1[j] * Sk
                Uvv = Pi * (2 * cv[2] * v1[j] ** 2 + dQ(xv[j]) * v2[j]) * Sk
                Uy = Pi * Qj * dS(xy[k]) * y1[k]
                Urv = dP(xr[i]) * r1[i] * dQ(xv[j]) * v1[j] * Sk
                Uijk = Pi * Qj * Sk
                want_r = z_rr * Urr + mu_r * Ur - rr * Uijk
                scale_r = abs(z_rr * Urr) + abs(mu_r * Ur) + abs(rr * Uijk) + 1e-300
                # v = v_max is an outflow face: the second-derivative term is not kept
                want_v = (z_vv * Uvv if j < nv - 1 else 0.0) + mu_v * Uv
                scale_v = abs(z_vv * Uvv) + abs(mu_v * Uv) + 1e-300
                want_y = mu_y * Uy
                scale_y = abs(mu_y * Uy) + 1e-300
                edge = i == 0 or j == 0 or j == nv - 1
                want_x = 0.0 if edge else z_rv * Urv
                scale_x = abs(z_rv * Urv) + 1e-300
                assert abs(A[0][k, j, i] - want_r) <= 1e-11 * scale_r, (i, j, k)
                assert abs(A[1][k, j, i] - want_v) <= 1e-11 * scale_v, (i, j, k)
                assert abs(A[2][k, j, i] - want_y) <= 1e-11 * scale_y, (i, j, k)
                assert abs(A[3][k, j, i] - want_x) <= 1e-11 * scale_x, (i, j, k)
                checked += 1
    assert checked == (nr - 1) * nv * (ny - 1)


def test_operators_second_order_on_smooth_physical_field():
    """U = exp(-a r) (1 + b v) exp(-c y) is not quadratic in the mesh coordinates;
    the interior error of each operator must fall like h^2."""
    errs = []
    for n in (17, 33, 65):
        p = _small_problem(n, n, n)
        r, _, _ = O.axis(p.axes[0])
        v, _, _ = O.axis(p.axes[1])
        y, _, _ = O.axis(p.axes[2])
        a, b, c = 8.0, 0.3, 40.0
        R, V, Y = np.meshgrid(r, v, y, indexing="ij")
        U = np.transpose(np.exp(-a * R) * (1 + b * V) * np.exp(-c * Y), (2, 1, 0)).copy()
        t = 1.0
        f, ft = O.forward(p, t), O.forward_dt(p, t)
        Ar = O.apply(p, 0, t, U)
        sl = (slice(1, -1), slice(1, -1), slice(1, -1))
        rr = r[None, None, :]
        vv = v[None, :, None]
        yy = y[:, None, None]
        z_rr = 0.5 * p.lam ** 2 * rr ** (2 * p.gamma) * vv
        mu_r = ft - p.kappa * (rr - f) + yy
        exact = z_rr * a * a * U + mu_r * (-a) * U - rr * U
        # restrict to the region the mesh resolves (r <= 0.2, v <= 5)
        mask = (rr <= 0.2) & (vv <= 5.0) & np.ones_like(yy, dtype=bool)
        errs.append(np.abs(Ar - exact)[sl][mask[sl]].max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.5, errs


def _dense_ops(p, t):
    shape = p.shape
    N = int(np.prod(shape))
    mats = []
    for d in range(4):
        M = np.zeros((N, N))
        e = np.zeros(N)
        for q in range(N):
            e[:] = 0.0
            e[q] = 1.0
            M[:, q] = O.apply(p, d, t, e.reshape(shape)).ravel()
        mats.append(M)
    return mats


def _dirichlet_mask(p):
    nr, nv, ny = (a.n for a in p.axes)
    mask = np.zeros(p.shape, dtype=bool)
    mask[:, :, nr - 1] = True
    mask[ny - 1, :, :] = True
    if p.axes[0].lo_face == O.DIRICHLET:
        mask[:, :, 0] = True
    return mask.ravel()


@pytest.mark.parametrize("kind", [W.CAPLET, W.BOND])
def test_douglas_step_factor_identity(kind):
    p = _small_problem(6, 5, 5)
    p.kind = kind
    n = 7
    dt = p.expiry / p.n_steps
    t_now, t_next, t_half = p.expiry - n * dt, p.expiry - (n + 1) * dt, p.expiry - (n + 0.5) * dt
    rng = np.random.default_rng(3)
    U0 = O.terminal(p) + 0.01 * rng.standard_normal(p.shape)
    U1 = O.step(p, n, U0.copy())
    Ar, Av, Ay, Ax = _dense_ops(p, t_half)
    I = np.eye(Ar.shape[0])
    th = 0.5
    Mr, Mv, My = I - th * dt * Ar, I - th * dt * Av, I - th * dt * Ay
    D0 = dt * (Ar + Av + Ay + Ax) @ U0.ravel()
    mask = _dirichlet_mask(p)
    r, _, _ = O.axis(p.axes[0])
    y, _, _ = O.axis(p.axes[2])
    g = lambda t: np.array([[[O.dirichlet(p, t, r[i], y[k]) for i in range(len(r))]
                             for _ in range(p.axes[1].n)] for k in range(len(y))]).ravel()
    D0[mask] = (g(t_next) - g(t_now))[mask]
    lhs = Mr @ Mv @ My @ (U1 - U0).ravel()
    assert np.abs(lhs - D0).max() <= 1e-13 * max(np.abs(D0).max(), 1e-300) + 1e-17
    # the wrong sweep order must not satisfy it (the factors do not commute)
    wrong = My @ Mv @ Mr @ (U1 - U0).ravel()
    assert np.abs(wrong - D0).max() > 1e3 * np.abs(lhs - D0).max()


def _unsplit_cn(p, n_steps):
    """Crank-Nicolson without splitting (dense solve), rho = 0, operators at t_{n+1/2}."""
    p.n_steps = n_steps
    dt = p.expiry / n_steps
    U = O.terminal(p).ravel()
    mask = _dirichlet_mask(p)
    r, _, _ = O.axis(p.axes[0])
    y, _, _ = O.axis(p.axes[2])
    g = lambda t: np.array([[[O.dirichlet(p, t, r[i], y[k]) for i in range(len(r))]
                             for _ in range(p.axes[1].n)] for k in range(len(y))]).ravel()
    I = np.eye(U.size)
    for n in range(n_steps):
        th = p.expiry - (n + 0.5) * dt
        Ar, Av, Ay, Ax = _dense_ops(p, th)
        A = Ar + Av + Ay + Ax
        rhs = dt * A @ U
        rhs[mask] = (g(p.expiry - (n + 1) * dt) - g(p.expiry - n * dt))[mask]
        U = U + np.linalg.solve(I - 0.5 * dt * A, rhs)
    return U


def test_douglas_splitting_error_is_second_order_without_mixed_term():
    p = _small_problem(6, 5, 5, rho=0.0)
    p.kind = W.BOND
    p.expiry = 1.0
    diffs = []
    for N in (4, 8, 16):
        p.n_steps = N
        ud = O.run(p).ravel()
        uc = _unsplit_cn(p, N)
        diffs.append(np.abs(ud - uc).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.0 < r1 < 5.5 and 3.3 < r2 < 4.8, diffs
