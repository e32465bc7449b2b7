"""GPU parity of the ADI schemes beyond the paper's Douglas step (Craig-Sneyd,
modified Craig-Sneyd, Hundsdorfer-Verwer, Douglas with Huang's
approximate-factorisation correction) and of Douglas with another theta,
against the CPU oracle on the same seeded inputs, through the C ABI.

Bar: as for Douglas, max|dU| / max|U| <= 1e-12 over the whole grid and
|dp| <= 1e-12 |p| for the price; both the fused explicit + r kernel and the
split pair run the correction stage.  Without a mixed term Craig-Sneyd is the
Douglas step bit for bit on the GPU too.
"""
import math

import numpy as np
import pytest

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hjm = pytest.importorskip("paper_1108_1688_amd.hjm")

REL = 1e-12
THETA_MCS = 1.0 / 3.0
THETA_HV = 0.5 + math.sqrt(3.0) / 6.0


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fused = hjm.get_r_fusion()
    minors = hjm.get_y_minors()
    yield
    hjm.set_r_fusion(fused)
    hjm.set_y_minors(minors)


def _spec(shape, steps, scheme, theta, rho=-0.6, kind=W.CAPLET, gaussian=False, af_iters=0):
    from dataclasses import replace
    m = W.ModelSpec(kappa=0.08, epsilon=0.45, rho=rho, **W.CURVE_SLOPED)
    k = W.atm_strike(m, 2.0, 3.0)
    s = W.SolveSpec(W.default_axes(*shape, k), m, W.PayoffSpec(kind, 2.0, 3.0, k), steps, m.f_level)
    if gaussian:
        s = W.gaussian_variant(s)
    return replace(s, scheme=scheme, theta=theta, af_iters=af_iters)


def _gpu(s):
    print(f"[gpu] shape={s.shape} steps={s.n_steps} scheme={s.scheme} theta={s.theta} af_iters={s.af_iters}",
          flush=True)
    g = hjm.Grid(s)
    plan = g.plan()
    g.step()
    p = g.price()
    U = g.solution().cpu().numpy().copy()
    g.close()
    return U, p, plan


def _check(s):
    Ug, pg, plan = _gpu(s)
    p = to_oracle(s)
    Uo = O.run(p, 0, s.n_steps)
    po = O.readout(p, Uo, s.r0, s.v0)
    assert np.isfinite(Ug).all()
    err = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    assert err <= REL, f"grid rel err {err:.3e}"
    assert abs(pg - po) <= REL * abs(po), (pg, po)
    return plan, err


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("scheme,theta", [(W.CS, 0.5), (W.MCS, THETA_MCS), (W.HV, THETA_HV), (W.DOUGLAS, 0.6)],
                         ids=["CS", "MCS", "HV", "Douglas-0.6"])
def test_scheme_parity(scheme, theta, path):
    hjm.set_r_fusion(path == "fused")
    plan, err = _check(_spec((64, 24, 32), 10, scheme, theta))
    assert plan["r_method"] == path and plan["yc_rows"] > 0
    assert plan["scheme"] == hjm.SCHEMES[scheme]
    print(f"scheme {scheme} theta {theta} {path}: grid rel err {err:.2e}")


@pytest.mark.parametrize("scheme,theta", [(W.CS, 0.5), (W.HV, THETA_HV)], ids=["CS", "HV"])
def test_scheme_ragged_tiles_and_faces(scheme, theta):
    """Several y planes per workgroup and ragged v / plane blocks (32 x 20 x
    16), and the Gaussian mode with both r faces Dirichlet (96 x 24 x 16)."""
    _check(_spec((32, 20, 16), 9, scheme, theta))
    _check(_spec((96, 24, 16), 24, scheme, theta, gaussian=True))


def test_cs_is_douglas_without_mixed_term_on_gpu():
    """With rho = 0 the corrections vanish and CS is Douglas, bit for bit:
    the correction schemes sweep y on stored pivots, so the Douglas grid
    takes them too (its default forms them in the sweep, equal to rounding)."""
    hjm.set_y_minors(False)
    U_d, p_d, _ = _gpu(_spec((64, 24, 32), 8, W.DOUGLAS, 0.5, rho=0.0))
    hjm.set_y_minors(True)
    U_c, p_c, _ = _gpu(_spec((64, 24, 32), 8, W.CS, 0.5, rho=0.0))
    assert np.array_equal(U_c, U_d) and p_c == p_d


def test_scheme_rejected_where_unsupported():
    """A grid whose r lines need the per-line chained solve (one long step)
    cannot run a correction scheme: HJM_EINVAL before any device work."""
    with pytest.raises(hjm.HjmError) as e:
        hjm.Grid(_spec((40, 24, 32), 1, W.CS, 0.5))
    assert e.value.status == hjm.EINVAL


@pytest.mark.parametrize("path", ["fused", "split"])
@pytest.mark.parametrize("q,theta", [(1, 0.5), (2, 0.5), (5, 0.5), (3, 0.6)])
def test_huang_parity(q, theta, path):
    """Douglas plus q Huang subiterations: the intermediate sweeps accumulate
    the iterate in place, the last adds it and its correction to U."""
    hjm.set_r_fusion(path == "fused")
    plan, err = _check(_spec((64, 24, 32), 8, W.HUANG, theta, af_iters=q))
    assert plan["r_method"] == path and plan["scheme"] == "huang"
    print(f"huang q={q} theta={theta} {path}: grid rel err {err:.2e}")


def test_huang_one_subiteration_is_hv_on_gpu():
    """One subiteration at theta = 1/2 is Hundsdorfer-Verwer at theta = 1/2:
    on the GPU the two run the same kernels with the same coefficients, so
    they agree bit for bit."""
    Uh, ph, _ = _gpu(_spec((64, 24, 32), 6, W.HUANG, 0.5, af_iters=1))
    Uv, pv, _ = _gpu(_spec((64, 24, 32), 6, W.HV, 0.5))
    assert np.array_equal(Uh, Uv) and ph == pv


@pytest.mark.parametrize("path", ["fused", "split"])
def test_batch_of_mixed_schemes_equals_single_grids(path):
    """A batch whose solves use different ADI schemes (each sweep sequence
    its own launch groups, the stage-2 descriptors after the stage-1 ones,
    uneven step counts so that the solves drop out at different steps):
    every price equals its own grid's bit for bit, the graph replay equals
    the eager run, and a CS and a Huang solve match the oracle's scheme."""
    hjm.set_r_fusion(path == "fused")
    specs = [_spec((64, 24, 32), 8, W.CS, 0.5), _spec((64, 24, 32), 6, W.MCS, THETA_MCS),
             _spec((64, 24, 32), 7, W.HV, THETA_HV), _spec((64, 24, 32), 5, W.HUANG, 0.5, af_iters=2),
             _spec((64, 24, 32), 8, W.DOUGLAS, 0.5), _spec((64, 24, 32), 4, W.DOUGLAS, 0.6),
             _spec((32, 24, 48), 6, W.CS, 0.5, kind=W.FLOORLET), _spec((64, 24, 32), 8, W.CS, 0.5, kind=W.FLOORLET)]
    print(f"[gpu] mixed-scheme batch of {len(specs)} ({path})", flush=True)
    st = torch.cuda.Stream()
    b = hjm.Batch(specs, stream=st)
    eager = b.run().prices()
    replay = b.run(graph=True).prices()
    again = b.run(graph=True).prices()
    n_ops = b.operators()
    b.close()
    assert np.array_equal(eager, replay) and np.array_equal(replay, again)
    # the CS caplet and floorlet on one mesh share an operator, nothing else does
    assert n_ops == len(specs) - 1
    for sp, pb in zip(specs, eager):
        _, pg, plan = _gpu(sp)
        assert plan["r_method"] == path
        assert pg == pb, (sp.scheme, sp.theta, pg, pb)
    for sp, pb in ((specs[0], eager[0]), (specs[3], eager[3])):
        p = to_oracle(sp)
        po = O.readout(p, O.run(p, 0, sp.n_steps), sp.r0, sp.v0)
        assert abs(pb - po) <= REL * abs(po), (sp.scheme, pb, po)


def test_batch_scheme_rejected_where_unsupported():
    """A batch with a correction scheme on a grid that needs the per-line
    chained r solve is refused before any device work, naming the solve."""
    specs = [_spec((64, 24, 32), 4, W.DOUGLAS, 0.5), _spec((40, 24, 32), 1, W.CS, 0.5)]
    with pytest.raises(hjm.HjmError) as e:
        hjm.Batch(specs)
    assert e.value.status == hjm.EINVAL and "solve 1" in str(e.value)
