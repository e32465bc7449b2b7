"""GPU behaviour of the C ABI: call-order errors, checkpoint / resume,
determinism, health flag, and the batched mode against single solves."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from adapt import to_oracle
from paper_1108_1688_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hjm = pytest.importorskip("paper_1108_1688_amd.hjm")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small():
    return W.with_shape(W.config1()[1], 40, 24, 20, 50)


def test_price_before_last_step_and_too_many_steps():
    s = small()
    g = hjm.Grid(s)
    g.step(10)
    with pytest.raises(hjm.HjmError) as e:
        g.price()
    assert e.value.status == hjm.ESTATE
    with pytest.raises(hjm.HjmError) as e:
        g.step(41)
    assert e.value.status == hjm.ESTATE
    g.step(40)
    assert 0.0 < g.price() < 1.0
    with pytest.raises(hjm.HjmError) as e:
        g.price(r0=3.0)
    assert e.value.status == hjm.EINVAL


def test_deterministic_bitwise():
    s = small()
    a = hjm.Grid(s).step()
    b = hjm.Grid(s).step()
    assert torch.equal(a.solution(), b.solution())
    assert a.price() == b.price()


def test_checkpoint_resume_bitwise():
    s = small()
    full = hjm.Grid(s).step()
    g = hjm.Grid(s)
    g.step(25)
    saved = g.solution().clone()
    g.step(25)
    # restore the checkpoint into a fresh handle and finish
    h = hjm.Grid(s)
    h.solution().copy_(saved)
    h.set_step(25)
    h.step(25)
    assert torch.equal(h.solution(), full.solution())
    assert h.price() == full.price()


def test_nan_in_grid_reports_numeric_error():
    s = small()
    g = hjm.Grid(s)
    g.step(5)
    g.solution()[3, 4, 5] = float("nan")
    g.step(45)
    with pytest.raises(hjm.HjmError) as e:
        g.price()
    assert e.value.status == hjm.ENUMERIC


def test_stream_argument_is_used():
    s = small()
    st = torch.cuda.Stream()
    g = hjm.Grid(s, stream=st)
    g.step()
    ref = hjm.Grid(s).step()
    assert g.price() == ref.price()


def _batch_specs():
    specs = W.config4(n=12, seed=7)
    # shrink most step counts so the test stays short (long steps put the r
    # lines on the chained solve); two keep theirs (split r solve); shapes stay
    # uneven, so the batch mixes every kernel variant
    from dataclasses import replace
    return [replace(sp, n_steps=max(3, sp.n_steps // 10)) for sp in specs[:10]] + specs[10:]


def test_batch_equals_single_solves_bitwise():
    specs = _batch_specs()
    b = hjm.Batch(specs).run()
    prices = b.prices()
    for sp, pb in zip(specs, prices):
        assert pb == hjm.Grid(sp).step().price()


def test_batch_graph_replays_match_eager():
    specs = _batch_specs()
    st = torch.cuda.Stream()
    eager = hjm.Batch(specs, stream=st).run(graph=False).prices()
    b = hjm.Batch(specs, stream=st)
    for rep in range(3):
        b.run(graph=True)
        got = b.prices()
        assert np.array_equal(got, eager), rep
        # eager work between replays
        x = torch.randn(1000, device="cuda") * 2
        torch.cuda.synchronize()
        del x


def test_batch_subset_against_oracle():
    specs = _batch_specs()[:4]
    prices = hjm.Batch(specs).run().prices()
    for sp, pg in zip(specs, prices):
        p = to_oracle(sp)
        po, _ = O.price(p, sp.r0, sp.v0)
        assert abs(pg - po) <= 1e-12 * abs(po), (pg, po)


def test_batch_profile_counts_and_prices():
    """Timing a batch's first steps changes no price; the points each pass
    reports are the grid points of the solves still running at those steps
    (the r pass only counts solves whose r lines have a kernel of their own)."""
    specs = _batch_specs()
    st = torch.cuda.Stream()
    plain = hjm.Batch(specs, stream=st).run().prices()
    k = 5
    b = hjm.Batch(specs, stream=st)
    b.profile(k)
    b.run()
    assert np.array_equal(b.prices(), plain)
    ms, n, pts = b.profile_read()
    split = [hjm.Grid(sp).plan()["r_method"] == "split" for sp in specs]
    total = sum(sp.points * min(k, sp.n_steps) for sp in specs)
    total_split = sum(sp.points * min(k, sp.n_steps) for sp, s in zip(specs, split) if s)
    assert pts[0] == pts[2] == pts[3] == total
    assert pts[1] == total_split
    for q in range(hjm.N_PASSES):
        assert (n[q] > 0) == (pts[q] > 0)
        assert n[q] <= k * len(specs)
        if n[q]:
            assert ms[q] > 0.0
    # the sums restart after a read; graph runs are never timed
    assert b.profile_read()[1] == [0] * hjm.N_PASSES
    b.run(graph=True)
    assert np.array_equal(b.prices(), plain)
    assert b.profile_read()[1] == [0] * hjm.N_PASSES


@pytest.mark.parametrize("lanes", [1, 3])
def test_batch_stream_lanes_bitwise(lanes):
    """Spreading the solves over stream lanes changes no bit, eager or from a
    graph, against the default (two lanes) and against single solves."""
    specs = _batch_specs()
    st = torch.cuda.Stream()
    ref = hjm.Batch(specs, stream=st).run().prices()
    old = hjm.get_batch_streams()
    try:
        hjm.set_batch_streams(lanes)
        b = hjm.Batch(specs, stream=st)
        assert np.array_equal(b.run().prices(), ref)
        for _ in range(2):
            b.run(graph=True)
            assert np.array_equal(b.prices(), ref)
    finally:
        hjm.set_batch_streams(old)
    for sp, p in list(zip(specs, ref))[::5]:
        assert p == hjm.Grid(sp).step().price()


def _rhs_specs(nv=24):
    """Right-hand sides of one operator (config 2's three strikes and an ATM
    floorlet on one 48 x nv x 32 mesh, 30 steps), a solve on another model, and
    two strikes on the discrete curve: three operators.  nv = 24: the v sweep
    on its own; nv = 32: folded into the other kernels (two 16-row segments),
    whose hand-over values each right-hand side keeps for itself."""
    from dataclasses import replace
    base = W.with_shape(W.config2()[1], 48, nv, 32, 30)
    k = base.payoff.strike
    same = [replace(base, payoff=replace(base.payoff, strike=k + dk)) for dk in (-0.01, 0.0, 0.01)]
    same.append(replace(base, payoff=replace(base.payoff, kind=W.FLOORLET)))
    other = replace(base, model=replace(base.model, epsilon=base.model.epsilon * 0.5))
    disc = W.with_shape(W.config_discrete()[0], 48, nv, 32, 30)
    disc2 = replace(disc, payoff=replace(disc.payoff, strike=disc.payoff.strike + 0.005))
    return [same[0], other, same[1], disc, same[2], disc2, same[3]]


@pytest.mark.parametrize("lanes,nv", [(1, 24), (2, 24), (1, 32), (3, 32)])
def test_shared_operator_batch_bitwise(lanes, nv):
    """Solves of one operator share tables (and stored y pivots; y tiles
    interleaved across the right-hand sides): prices equal the single grids'
    and the unshared batch's bit for bit, with the v sweep on its own and
    folded."""
    specs = _rhs_specs(nv)
    g = hjm.Grid(specs[0])
    assert g.plan()["v_fold"] == (nv == 32)
    g.close()
    old_l, old_s = hjm.get_batch_streams(), hjm.get_batch_share()
    try:
        hjm.set_batch_streams(lanes)
        hjm.set_batch_share(True)
        b = hjm.Batch(specs).run()
        shared, ops = b.prices(), b.operators()
        b.close()
        hjm.set_batch_share(False)
        b = hjm.Batch(specs).run()
        plain, ops_off = b.prices(), b.operators()
        b.close()
    finally:
        hjm.set_batch_streams(old_l)
        hjm.set_batch_share(old_s)
    assert ops == 3 and ops_off == len(specs)
    assert np.array_equal(shared, plain)
    for sp, pb in zip(specs, shared):
        g = hjm.Grid(sp).step()
        assert pb == g.price()
        g.close()
    po, _ = O.price(to_oracle(specs[4]), specs[4].r0, specs[4].v0)
    assert abs(shared[4] - po) <= 1e-12 * abs(po)


def test_shared_operator_graph_replays():
    specs = _rhs_specs()
    st = torch.cuda.Stream()
    eager = hjm.Batch(specs, stream=st).run(graph=False).prices()
    b = hjm.Batch(specs, stream=st)
    for rep in range(3):
        b.run(graph=True)
        assert np.array_equal(b.prices(), eager), rep
        x = torch.randn(1000, device="cuda") * 2
        torch.cuda.synchronize()
        del x
    b.close()


def config4_oracle_subset(specs, n=32):
    """Solves of the calibration workload to check against the oracle: for
    each axis and each of its sizes {32, 48, 64, 96} the cheapest solve with
    that size, the cheapest and the longest of the 200-step-class solves, the
    cheapest and the longest 96^3 solves, then the cheapest others up to n."""
    cost = [sp.points * sp.n_steps for sp in specs]
    chosen = []

    def add(q):
        if q not in chosen:
            chosen.append(q)

    for ax in range(3):
        for size in (32, 48, 64, 96):
            add(min((q for q in range(len(specs)) if specs[q].axes[ax].n == size), key=lambda q: cost[q]))
    longest = max(sp.n_steps for sp in specs)
    steps_max = [q for q in range(len(specs)) if specs[q].n_steps == longest]
    add(min(steps_max, key=lambda q: cost[q]))
    add(max(steps_max, key=lambda q: cost[q]))
    cubes = [q for q in range(len(specs)) if specs[q].points == 96 ** 3]
    add(min(cubes, key=lambda q: cost[q]))
    add(max(cubes, key=lambda q: cost[q]))
    for q in sorted(range(len(specs)), key=lambda q: cost[q]):
        if len(chosen) >= n:
            break
        add(q)
    return chosen


def test_config4_full_batch_against_single_grids_and_oracle():
    """The whole calibration workload as the bench times it (512 uneven
    solves, one batch replayed from a HIP graph): the graph replay equals an
    eager run bit for bit; every price equals its own single-grid solve
    (hjm_grid_create + hjm_adi_step + hjm_price) bit for bit and lies between 0
    and the discount factor; 32 solves covering every size on every axis, the
    longest step counts and the largest grids equal the oracle's to 1e-12."""
    specs = W.config4()
    st = torch.cuda.Stream()
    b = hjm.Batch(specs, stream=st)
    b.run(graph=True)
    graph = b.prices()
    b.run(graph=False)
    eager = b.prices()
    b.close()
    assert np.array_equal(graph, eager)
    assert np.all(np.isfinite(graph))
    methods = {}
    for q, (sp, pg) in enumerate(zip(specs, graph)):
        assert 0.0 <= pg <= O.discount(to_oracle(sp), sp.payoff.expiry) * (1 + 1e-12), (sp.shape, pg)
        g = hjm.Grid(sp, stream=st)
        plan = g.plan()
        g.step()
        single = g.price()
        g.close()
        assert single == pg, (q, sp.shape, single, pg)
        methods[q] = (plan["r_method"], plan["vs_rows"] > 0, plan["yc_rows"] > 0)
    subset = config4_oracle_subset(specs)
    print(f"config4 plans: {sorted(set(methods.values()))}; oracle subset plans: "
          f"{sorted(set(methods[q] for q in subset))}", flush=True)
    worst = 0.0
    for q in subset:
        sp = specs[q]
        po, _ = O.price(to_oracle(sp), sp.r0, sp.v0)
        err = abs(graph[q] - po) / abs(po)
        worst = max(worst, err)
        assert err <= 1e-12, (q, sp.shape, sp.n_steps, graph[q], po)
    print(f"config4 oracle subset: {len(subset)} solves, worst price rel err {worst:.2e}", flush=True)
