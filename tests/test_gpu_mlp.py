"""Surrogate MLP on the GPU (through the C ABI) against its CPU oracle, and
what the trained network gains over the solver alone.

Bars.  The GPU and the oracle round to BF16 at the same points; they differ
only in how the FP32 (GPU) and float64 (oracle) sums of BF16 products round,
about 1e-6 relative, which can flip the BF16 rounding of an activation lying
that close to a rounding boundary (one BF16 unit, 2^-8 relative, in a few
elements per 10^4), and the flips propagate through the later layers.  The
size of that effect is measured, not assumed: the oracle's float32-sum
variant (emulate32) differs from its float64-sum variant by the same
mechanism, and the GPU must stay within three times that distance (plus
1e-5 of the output scale); a wrong layout or index would miss it by orders
of magnitude.  Gradient tensors agree per tensor in relative L2 norm within
four times the same spread of the oracle's gradients (the GPU also sums the
backward products in float32), plus 2e-5; box flags are compared exactly
(both sides compare the same float32 values).
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1108_1688_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hjm = pytest.importorskip("paper_1108_1688_amd.hjm")
S = pytest.importorskip("paper_1108_1688_amd.surrogate")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


LO, HI = W.SURROGATE_BOX_LO, W.SURROGATE_BOX_HI


def _rows(n, seed, outside=0):
    x = W.surrogate_params(n, seed)
    if outside:
        x[:outside] = W.surrogate_outside(outside, seed + 1)
    return x.astype(np.float32)


def _params(seed):
    p = S.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    b = M.unpack(p)
    for l in (1, 2, 3, 4):
        b[f"b{l}"][:] = 0.1 * rng.standard_normal(256)
    b["b5"][:] = 0.3
    return M.pack(b).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_forward_and_box_flags_match_oracle():
    p = _params(1)
    x = _rows(300, 2, outside=40)  # 300: a ragged tail of the 64-row tiles
    m = S.make_mlp(max_batch=128, baseline=False)   # several passes of max_batch rows
    m.set_params(p)
    y, inb = m.infer(_dev(x))
    y = y.cpu().numpy().astype(np.float64)
    yo, c = M.forward(p.astype(np.float64), x, LO, HI, emulate=True)
    yo = yo * S.PLAIN_SCALE
    assert np.array_equal(inb.cpu().numpy().astype(bool), c["inside"])
    assert c["inside"].sum() == 260
    y32, _ = M.forward(p.astype(np.float64), x, LO, HI, emulate="emulate32")
    y32 = y32 * S.PLAIN_SCALE
    scale = np.abs(yo).mean()
    err = np.abs(y - yo) / scale
    ref = np.abs(y32 - yo) / scale
    print(f"forward err / mean |y|: max {err.max():.2e} rms {np.sqrt(np.mean(err**2)):.2e}; "
          f"oracle fp32-vs-fp64 sums: max {ref.max():.2e} rms {np.sqrt(np.mean(ref**2)):.2e}")
    assert err.max() <= 3 * ref.max() + 1e-5
    assert np.sqrt(np.mean(err ** 2)) <= 3 * np.sqrt(np.mean(ref ** 2)) + 1e-5


def test_baseline_output_and_targets_match_oracle():
    """With the Gaussian caplet baseline: the reported price is B exp(0.1 y)
    with y the network (same bar as the plain forward, on the recovered y),
    and the targets are 10 ln(price / B), both against the oracle's own
    baseline; a non-positive price gives NaN; invalid constants are refused."""
    p = _params(1)
    x = _rows(300, 2)
    x64 = x.astype(np.float64)
    m = S.make_mlp(max_batch=128)
    m.set_params(p)
    y, inb = m.infer(_dev(x))
    assert inb.cpu().numpy().all()
    y = y.cpu().numpy().astype(np.float64)
    yo, _ = M.forward(p.astype(np.float64), x, LO, HI, emulate=True)
    y32, _ = M.forward(p.astype(np.float64), x, LO, HI, emulate="emulate32")
    B = M.caplet_baseline(x64, *S.GAUSS_ARGS)
    assert np.all(B > 0) and np.all(np.isfinite(y)) and np.all(y > 0)
    yb = np.log(y / B) / S.OUT_SCALE  # the GPU's network output, recovered
    scale = np.abs(yo).mean()
    err = np.abs(yb - yo) / scale
    ref = np.abs(y32 - yo) / scale
    print(f"baseline forward err / mean |y|: max {err.max():.2e}; oracle fp32-vs-fp64 sums: max {ref.max():.2e}")
    # the price is stored as float32: 6e-8 relative, 6e-7 in network units
    assert err.max() <= 3 * ref.max() + 1e-5 + 1e-6 / scale
    price = B * np.exp(np.random.default_rng(9).uniform(-1.0, 2.0, len(x)))
    price[:3] = (0.0, -1e-6, 1.0)
    t = m.targets(_dev(x), torch.from_numpy(price).cuda()).cpu().numpy().astype(np.float64)
    to = M.baseline_target(x64[3:], price[3:], S.OUT_SCALE, 0.0, S.GAUSS_ARGS)
    assert np.isnan(t[0]) and np.isnan(t[1])
    np.testing.assert_allclose(t[3:], to, rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(np.exp(-S.OUT_SCALE * t[2]), B[2], rtol=1e-6)
    with pytest.raises(hjm.HjmError):
        m.set_baseline(0.15, 1.5, 0.25, 0.5, 1.0)
    with pytest.raises(hjm.HjmError):
        m.set_baseline(0.15, 0.9, 0.25, 0.0, 1.0)
    # without the baseline the targets are the scaled prices
    m.clear_baseline()
    t = m.targets(_dev(x[3:]), torch.from_numpy(price[3:]).cuda()).cpu().numpy()
    np.testing.assert_allclose(t, (price[3:] / S.OUT_SCALE).astype(np.float32), rtol=1e-6)
    m.close()


def test_gradients_and_loss_match_oracle():
    p = _params(3)
    n = 700  # spans several 256-row gradient chunks, with a tail
    x = _rows(n, 4)
    t = np.random.default_rng(5).standard_normal(n).astype(np.float32)
    m = S.make_mlp(max_batch=1024)
    m.set_params(p)
    sse = m.gradients(_dev(x), _dev(t))
    g = m.grads().astype(np.float64)
    so, go = M.loss_and_grads(p.astype(np.float64), x, t, LO, HI, emulate=True)
    s32, g32 = M.loss_and_grads(p.astype(np.float64), x, t, LO, HI, emulate="emulate32")
    assert abs(sse - so) <= 3 * abs(s32 - so) + 1e-6 * so
    G, Go, G32 = M.unpack(g), M.unpack(go), M.unpack(g32)
    for name, _ in M.SHAPES:
        norm = max(np.linalg.norm(Go[name]), 1e-30)
        rel = np.linalg.norm(G[name] - Go[name]) / norm
        # the oracle's own spread between float32 and float64 layer sums (the
        # GPU also sums the backward products in float32, hence 4x)
        spread = np.linalg.norm(G32[name] - Go[name]) / norm
        print(f"{name}: rel L2 err {rel:.2e} (oracle fp32-vs-fp64 sums {spread:.2e})")
        assert rel <= 4 * spread + 2e-5, name


def test_adam_step_matches_oracle():
    p = _params(6)
    x = _rows(256, 7)
    t = np.random.default_rng(8).standard_normal(256).astype(np.float32)
    m = S.make_mlp(max_batch=256)
    m.set_params(p)
    m.gradients(_dev(x), _dev(t))
    g = m.grads().astype(np.float64)
    m.adam(1e-3)
    got = m.params().astype(np.float64)
    want, _, _ = M.adam_step(p.astype(np.float64), np.zeros_like(g), np.zeros_like(g), g, 1, 1e-3)
    assert np.abs(got - want).max() <= 1e-6


# relative-error bars of the small training run below (3072 rows, 150
# epochs): about twice the values measured on the GPU (median 9.9e-3, p95
# 0.105)
MED_BAR, P95_BAR = 2e-2, 2e-1


def test_trained_surrogate_gains_over_the_solver():
    """Train on solver prices; on new rows in the box the surrogate prices
    far faster than the solver, with a stated error; rows outside the box
    are priced by the solver itself."""
    torch.manual_seed(0)
    x, prices = S.training_set(192, seed=11)  # 3072 rows
    m = S.make_mlp(max_batch=4096)
    m.set_params(S.init_params(12))
    res = S.fit(m, x, prices, epochs=150, batch=256, lr=2e-3, lr_final=2e-4, seed=13)
    assert res.losses[-1] < 0.1 * res.losses[0]
    # 512 validation rows: 32 solves, each read out at 16 values of v0 (the
    # solver's cost of these prices is these 32 batched solves)
    import time
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xv, pv = S.training_set(32, seed=14)
    torch.cuda.synchronize()
    adi_s = time.perf_counter() - t2
    S.training_set(32, seed=14)
    torch.cuda.synchronize()
    adi_s = min(adi_s, time.perf_counter() - t2 - adi_s)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    xd = _dev(xv)
    t0.record()
    y, inb = m.infer(xd)
    t1.record()
    torch.cuda.synchronize()
    surrogate_s = t0.elapsed_time(t1) * 1e-3
    ys = y.cpu().numpy().astype(np.float64)
    assert inb.cpu().numpy().all()
    err = np.abs(ys - pv)
    rms = float(np.sqrt(np.mean(err ** 2)))
    base = float(np.sqrt(np.mean((pv - prices.mean()) ** 2)))  # predicting the mean price
    big = pv > S.FIT_PRICE_FLOOR
    rel = err[big] / pv[big]
    med, p95 = float(np.median(rel)), float(np.percentile(rel, 95))
    print(f"surrogate rms {rms:.2e} (mean-price baseline {base:.2e}), relative error above "
          f"{S.FIT_PRICE_FLOOR:g}: median {med:.2e}, p95 {p95:.2e}, max {rel.max():.2e}; below it max abs "
          f"{err[~big].max() if (~big).any() else 0.0:.2e}; {len(xv) / surrogate_s:.3g} vs "
          f"{len(xv) / adi_s:.3g} prices/s")
    assert rms < 0.1 * base
    assert med <= MED_BAR and p95 <= P95_BAR, (med, p95)
    assert surrogate_s * 20 < adi_s
    # out of the box: solver prices, equal to a direct solve
    xo = W.surrogate_outside(6, 15).astype(np.float32)
    pr = S.price(m, xo)
    assert pr.n_fallback == 6 and not pr.in_box.any()
    assert np.array_equal(pr.prices, S.adi_prices(xo.astype(np.float64)))
