"""Autotuner: selection logic (host only) and, on a GPU, per-shape tiles
that a batch applies, with the tuned solves against the oracle."""
import numpy as np
import pytest

from paper_1108_1688_amd import workloads as W


def test_line_shapes_of_a_grid():
    from paper_1108_1688_amd import autotune as A
    assert A.line_shapes((96, 48, 32)) == [(0, 96, 48 * 32), (1, 48, 96 * 32), (2, 32, 96 * 48)]


def test_choose_takes_each_line_shapes_fastest_candidate():
    from paper_1108_1688_amd import autotune as A
    times = {(0, 96, 1536): {8: 30.0, 16: 25.0, 32: 28.0},
             (1, 48, 3072): {8: 20.0, 16: 22.0, 32: 18.0},
             (2, 32, 4608): {8: 9.0, 16: 11.0, 32: 10.0}}
    assert A.choose(times) == {(0, 96, 1536): 16, (1, 48, 3072): 32, (2, 32, 4608): 8}


def test_choose_per_axis_sums_each_axis_over_its_line_shapes():
    from paper_1108_1688_amd import autotune as A
    times = {(0, 96, 1536): {8: 30.0, 16: 25.0, 32: 28.0},
             (0, 64, 2048): {8: 10.0, 16: 16.0, 32: 12.0},   # r: 8 -> 40, 16 -> 41, 32 -> 40
             (1, 48, 3072): {8: 20.0, 16: 22.0, 32: 18.0},
             (2, 32, 4608): {8: 9.0, 16: 11.0, 32: 10.0}}
    got = A.choose_per_axis(times)
    assert got == {(0, 96, 1536): 8, (0, 64, 2048): 8, (1, 48, 3072): 32, (2, 32, 4608): 8}
    # a candidate missing on one of the axis's shapes is not eligible for that axis
    times[(2, 48, 100)] = {16: 1.0, 32: 1.0}
    got = A.choose_per_axis(times)
    assert got[(2, 32, 4608)] == 32 and got[(2, 48, 100)] == 32


def test_weigh_sums_the_work_of_every_grid_shape_with_the_line_shape():
    from paper_1108_1688_amd import autotune as A
    # the r lines of (32, 96, 64) and (32, 64, 96) are one line shape
    shapes = {(32, 96, 64): (None, 0.25), (32, 64, 96): (None, 0.5), (48, 48, 48): (None, 0.25)}
    raw = {k: {8: 1.0, 16: 2.0} for sh in shapes for k in A.line_shapes(sh)}
    w = A.weigh(raw, shapes)
    assert w[(0, 32, 6144)] == {8: 0.75, 16: 1.5}
    assert w[(1, 96, 2048)] == {8: 0.25, 16: 0.5}
    assert w[(2, 48, 2304)] == {8: 0.25, 16: 0.5}
    assert len(w) == 8


def test_workload_key_depends_on_shapes_steps_and_tile():
    from paper_1108_1688_amd import autotune as A
    specs = W.config4(16)
    k = A.workload_key(specs, (16, 16, 16))
    assert k == A.workload_key(list(specs), (16, 16, 16))
    assert k != A.workload_key(specs, (8, 16, 16))
    assert k != A.workload_key(specs[:-1], (16, 16, 16))


def test_shapes_by_work_weights_sum_to_one():
    from paper_1108_1688_amd import autotune as A
    specs = W.config4(64)
    shapes = A.shapes_by_work(specs)
    total = sum(s.points * s.n_steps for s in specs)
    assert abs(sum(w for _, w in shapes.values()) - 1.0) < 1e-12
    for sh, (spec, w) in shapes.items():
        assert spec.shape[::-1] == sh
        mine = sum(s.points * s.n_steps for s in specs if s.shape[::-1] == sh)
        assert abs(w - mine / total) < 1e-12
        assert spec.n_steps == max(s.n_steps for s in specs if s.shape[::-1] == sh)


def test_axis_tile_overrides_round_trip_and_refusals():
    from paper_1108_1688_amd import hjm
    hjm.clear_axis_tiles()
    hjm.set_axis_tile(1, 48, 0, 32)
    hjm.set_axis_tile(2, 96, 96 * 64, 8)
    assert hjm.get_axis_tile(1, 48) == 32 and hjm.get_axis_tile(2, 96, 96 * 64) == 8
    assert hjm.get_axis_tile(2, 96) == 0
    for bad in ((3, 48, 0, 16), (0, 4, 0, 16), (0, 48, 0, 12), (0, 48, -1, 16)):
        with pytest.raises(hjm.HjmError):
            hjm.set_axis_tile(*bad)
    hjm.set_axis_tile(1, 48, 0, 0)
    assert hjm.get_axis_tile(1, 48) == 0
    hjm.clear_axis_tiles()
    assert hjm.get_axis_tile(2, 96, 96 * 64) == 0


@pytest.mark.gpu
def test_tuned_batch_matches_oracle_and_untuned(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle as O
    from adapt import to_oracle
    from paper_1108_1688_amd import autotune as A
    from paper_1108_1688_amd import hjm
    old = hjm.get_line_tile()
    old_lanes = hjm.get_batch_streams()
    base = W.config2()[1]
    specs = [W.with_shape(base, 64, 48, 32, 30), W.with_shape(base, 96, 32, 64, 24),
             W.with_shape(base, 32, 64, 48, 20)]
    try:
        hjm.clear_axis_tiles()
        untuned = hjm.Batch(specs).run().prices()
        cache = str(tmp_path / "tune.json")
        t = A.tune(specs, steps=3, cache=cache)
        assert not t.cached and t.timed_grids == 3 * len(A.CANDIDATES)
        assert len(t.per_shape) == 9 and len(t.per_axis) == 9
        assert set(t.batch_ms) == {"default", "per_axis", "per_shape"}
        assert t.batch_ms[t.chosen] == min(t.batch_ms.values())
        assert t.choice == {"default": {}, "per_axis": t.per_axis, "per_shape": t.per_shape}[t.chosen]
        assert set(t.lanes_ms) == set(A.LANES) and t.lanes_ms[t.lanes] == min(t.lanes_ms.values())
        assert hjm.get_batch_streams() == t.lanes
        assert tuple(hjm.get_line_tile()) == tuple(old)
        for (axis, n, lines), rows in t.per_shape.items():
            assert hjm.get_axis_tile(axis, n, lines) == t.choice.get((axis, n, lines), 0)
        print(f"tuned: {t.summary()}")
        again = A.tune(specs, cache=cache)
        assert again.cached and again.choice == t.choice and again.chosen == t.chosen and again.lanes == t.lanes
        assert again.us == t.us
        # per-kernel times are kept per line shape: a batch of two of these
        # grid shapes times no grid at all (only its end-to-end choice)
        import json
        stored = json.load(open(cache))
        assert sum(1 for k in stored if k.startswith("line:")) == 9
        part = A.tune(specs[:2], cache=cache, apply=False)
        assert not part.cached and part.timed_grids == 0 and len(part.per_shape) == 6
        tuned = hjm.Batch(specs).run().prices()
        # every proposal, installed, against the oracle and single grids
        for ov in (t.per_shape, t.per_axis):
            hjm.clear_axis_tiles()
            for (axis, n, lines), rows in ov.items():
                hjm.set_axis_tile(axis, n, lines, rows)
            pb_all = hjm.Batch(specs).run().prices()
            for sp, pb in zip(specs, pb_all):
                g = hjm.Grid(sp)
                g.step()
                assert g.price() == pb
                g.close()
        for sp, pb, pu in zip(specs, tuned, untuned):
            po, _ = O.price(to_oracle(sp), sp.r0, sp.v0)
            assert abs(pb - po) <= 1e-12 * abs(po)
            assert abs(pu - po) <= 1e-12 * abs(po)
    finally:
        hjm.clear_axis_tiles()
        hjm.set_line_tile(*old)
        hjm.set_batch_streams(old_lanes)
