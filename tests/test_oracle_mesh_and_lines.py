"""Pins of the oracle's sinh mesh (section 4.3 / 7.1) and tridiagonal line solver
(section 5): Jacobians against finite differences of the map itself, the
inverse map, and line solves against a dense LU (numpy.linalg.solve)."""
import numpy as np
import pytest

import oracle as O
from paper_1108_1688_amd import workloads as W

AXES = [O.Axis(65, 0.0, 2.5, 0.03, 0.005), O.Axis(65, 0.0, 30.0, 0.5, 0.5),
        O.Axis(65, 0.0, 0.025, 0.0, 5e-5), O.Axis(65, -0.5, 2.5, 0.02, 0.005)]


@pytest.mark.parametrize("ax", AXES)
def test_mesh_ends_monotone_and_clustered(ax):
    z, J, J2 = O.axis(ax)
    assert z[0] == ax.z_min and z[-1] == ax.z_max
    assert np.all(np.diff(z) > 0)
    assert np.all(J > 0)
    # finer spacing next to the centre than at the far end
    c = int(np.argmin(np.abs(z - ax.center)))
    c = min(max(c, 1), len(z) - 2)
    assert (z[c + 1] - z[c]) < (z[-1] - z[-2])


@pytest.mark.parametrize("ax", AXES)
def test_jacobians_match_differences_of_the_map(ax):
    """J = dz/dx and J2 = d2z/dx2: Richardson-extrapolated central differences of
    z itself, taken on a 32x finer mesh (steps h/32 and h/16)."""
    n = ax.n
    fine = O.Axis(32 * (n - 1) + 1, ax.z_min, ax.z_max, ax.center, ax.alpha)
    zf, _, _ = O.axis(fine)
    hf = 1.0 / (fine.n - 1)
    _, J, J2 = O.axis(ax)
    for m in range(1, n - 1):
        q = 32 * m
        d1a = (zf[q + 1] - zf[q - 1]) / (2 * hf)
        d1b = (zf[q + 2] - zf[q - 2]) / (4 * hf)
        d2a = (zf[q + 1] - 2 * zf[q] + zf[q - 1]) / hf ** 2
        d2b = (zf[q + 2] - 2 * zf[q] + zf[q - 2]) / (2 * hf) ** 2
        d1 = (4 * d1a - d1b) / 3
        d2 = (4 * d2a - d2b) / 3
        assert J[m] == pytest.approx(d1, rel=1e-7)
        assert J2[m] == pytest.approx(d2, rel=1e-4, abs=1e-6 * abs(J[m]))


@pytest.mark.parametrize("ax", AXES)
def test_inverse_map_round_trip(ax):
    z, _, _ = O.axis(ax)
    h = 1.0 / (ax.n - 1)
    for m in range(ax.n):
        assert O.axis_x(ax, z[m]) == pytest.approx(m * h, abs=1e-12)


def _dense(a, b, c, e_lo, e_hi):
    n = len(b)
    M = np.zeros((n, n))
    for m in range(n):
        M[m, m] = b[m]
        if m > 0:
            M[m, m - 1] = a[m]
        if m < n - 1:
            M[m, m + 1] = c[m]
    M[0, 2] += e_lo
    M[n - 1, n - 3] += e_hi
    return M


@pytest.mark.parametrize("n", [4, 5, 7, 32, 129])
@pytest.mark.parametrize("kind", ["interior", "outflow", "dirichlet", "advection"])
def test_line_solve_matches_dense_lu(n, kind):
    rng = np.random.default_rng(n * 7 + len(kind))
    a = -rng.uniform(0.0, 1.0, n)
    c = -rng.uniform(0.0, 1.0, n)
    b = 1.0 + np.abs(a) + np.abs(c) + rng.uniform(0.0, 0.5, n)
    e_lo = e_hi = 0.0
    if kind == "outflow":
        # one-sided rows: (-3,4,-1) pattern scaled, diagonal >= 1
        s = rng.uniform(0.1, 2.0)
        b[0], c[0], e_lo = 1 + 1.5 * s, -2 * s, 0.5 * s
        s = rng.uniform(0.1, 2.0)
        b[-1], a[-1], e_hi = 1 + 1.5 * s, -2 * s, 0.5 * s
    elif kind == "dirichlet":
        for m in (0, n - 1):
            a[m], b[m], c[m] = 0.0, 1.0, 0.0
    elif kind == "advection":
        # pure first-derivative rows (y direction): I + skew part
        beta = rng.uniform(-0.4, 0.4, n)
        a, b, c = -beta, np.ones(n), beta.copy()
        s = rng.uniform(0.0, 1.0)
        b[0], c[0], e_lo = 1 + 1.5 * s, -2 * s, 0.5 * s
        a[-1], b[-1], c[-1] = 0.0, 1.0, 0.0
    a[0] = 0.0
    c[-1] = 0.0
    d = rng.standard_normal(n)
    x = O.line_solve(a, b, c, e_lo, e_hi, d)
    ref = np.linalg.solve(_dense(a, b, c, e_lo, e_hi), d)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_readout_exact_on_cubics_and_at_nodes():
    """4-point Lagrange readout in (x_r, x_v) on the lowest y plane is exact for
    fields cubic in each mesh coordinate and returns node values at nodes."""
    import adapt
    s = W.with_shape(W.config1()[1], 21, 17, 5)
    p = adapt.to_oracle(s)
    nr, nv, ny = 21, 17, 5
    xr = np.arange(nr) / (nr - 1)
    xv = np.arange(nv) / (nv - 1)
    cub = lambda x, c: c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
    cr, cv = [0.3, -1.2, 2.0, 0.7], [1.1, 0.4, -0.9, 0.25]
    U = np.zeros((ny, nv, nr))
    U[0] = cub(xv, cv)[:, None] * cub(xr, cr)[None, :]
    U[1:] = 1e3  # planes above y_min must not contribute
    for r0, v0 in [(0.0, 0.0), (0.031, 1.0), (0.2, 3.7), (2.5, 30.0), (1e-4, 29.0)]:
        ar = O.axis_x(p.axes[0], r0)
        av = O.axis_x(p.axes[1], v0)
        want = cub(ar, cr) * cub(av, cv)
        assert O.readout(p, U, r0, v0) == pytest.approx(want, rel=1e-12, abs=1e-12)
    z, _, _ = O.axis(p.axes[0])
    v, _, _ = O.axis(p.axes[1])
    rng = np.random.default_rng(1)
    R = rng.standard_normal((ny, nv, nr))
    for i, j in [(0, 0), (5, 3), (20, 16), (10, 8)]:
        assert O.readout(p, R, z[i], v[j]) == pytest.approx(R[0, j, i], rel=1e-12, abs=1e-13)
