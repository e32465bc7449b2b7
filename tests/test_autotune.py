"""Autotuner: selection logic (host only) and, on a GPU, a tuned solve."""
import numpy as np
import pytest

from paper_1108_1688_amd import workloads as W


def test_choose_takes_each_kernels_best_value():
    from paper_1108_1688_amd import autotune as A
    runs = [{"setting": (8, 8, 8, 4), "us": [30.0, 50.0, 20.0, 40.0]},
            {"setting": (16, 16, 16, 8), "us": [25.0, 35.0, 22.0, 33.0]},
            {"setting": (32, 32, 32, 16), "us": [28.0, 36.0, 18.0, 35.0]}]
    setting, per = A.choose(runs, split=True)
    assert setting == (16, 32, 16, 8)
    assert per == {"explicit": 25.0, "r": 35.0, "v": 18.0, "y+update": 33.0}


def test_choose_fused_r_follows_the_explicit_pass():
    from paper_1108_1688_amd import autotune as A
    from paper_1108_1688_amd import hjm
    runs = [{"setting": (8, 8, 8, 4), "us": [90.0, 0.0, 20.0, 40.0]},
            {"setting": (16, 16, 16, 8), "us": [80.0, 0.0, 22.0, 33.0]},
            {"setting": (32, 32, 32, 16), "us": [95.0, 0.0, 18.0, 35.0]}]
    setting, _ = A.choose(runs, split=False)
    assert setting[:3] == (16, 32, 16) and setting[3] == hjm.get_explicit_chunk()


def test_representatives_weights_sum_to_one_and_prefer_big_work():
    from paper_1108_1688_amd import autotune as A
    specs = W.config4(64)
    reps = A.representatives(specs, k=3)
    assert len(reps) == 3
    work = {}
    for s in specs:
        sh = s.shape
        work[sh] = work.get(sh, 0) + s.points * s.n_steps
    top = sorted(work.values(), reverse=True)[:3]
    assert np.allclose([w for _, w in reps], [t / sum(work.values()) for t in top])


@pytest.mark.gpu
def test_tuned_solve_matches_oracle(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle as O
    from adapt import to_oracle
    from paper_1108_1688_amd import autotune as A
    from paper_1108_1688_amd import hjm
    old = hjm.get_line_tile(), hjm.get_explicit_chunk()
    try:
        s = W.with_shape(W.config2()[1], 64, 48, 32, 30)
        cache = str(tmp_path / "tune.json")
        t = A.tune([s], steps=3, cache=cache)
        assert len(t.runs) == len(A.DIAGONAL) and not t.cached
        assert (hjm.get_line_tile() + (hjm.get_explicit_chunk(),)) == t.setting
        again = A.tune([s], cache=cache)
        assert again.cached and again.setting == t.setting
        g = hjm.Grid(s)
        g.step()
        pg = g.price()
        Ug = g.solution().cpu().numpy().copy()
        g.close()
        p = to_oracle(s)
        Uo = O.run(p, 0, s.n_steps)
        assert np.abs(Ug - Uo).max() <= 1e-12 * np.abs(Uo).max()
        po = O.readout(p, Uo, s.r0, s.v0)
        assert abs(pg - po) <= 1e-12 * abs(po)
    finally:
        hjm.set_line_tile(*old[0])
        hjm.set_explicit_chunk(old[1])
