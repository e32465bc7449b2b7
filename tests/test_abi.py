"""C-ABI checks that need no GPU: the library loads, exports every function
include/hjm.h declares, and rejects invalid problems on the host before any
device work (validation runs first, so no HIP call is made)."""
import ctypes as C
import os
import re
from dataclasses import replace

import pytest

from paper_1108_1688_amd import hjm
from paper_1108_1688_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hjm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|hjm_status)\s+(hjm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hjm.LIB_PATH):
        from paper_1108_1688_amd import build
        build.build()
    return hjm.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 15, names
    raw = C.CDLL(hjm.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_status_strings(L):
    for code in (hjm.OK, hjm.EINVAL, hjm.ENOMEM, hjm.EDEVICE, hjm.ENUMERIC, hjm.ESTATE):
        assert L.hjm_status_str(code).decode().startswith("HJM_")
    assert L.hjm_status_str(-99).decode() == "unknown hjm_status"


def _create(spec, ws_ptr=0x100000, ws_bytes=1 << 40):
    L = hjm.lib()
    h = C.c_void_p()
    ax = hjm.make_axes(spec.axes)
    m = hjm.make_model(spec.model)
    p = hjm.make_payoff(spec.payoff)
    st = L.hjm_grid_create(ax, C.byref(m), C.byref(p), spec.n_steps, C.c_void_p(ws_ptr), ws_bytes,
                           C.c_void_p(0), C.byref(h))
    return st, L.hjm_last_error().decode()


def test_workspace_bytes(L):
    s = W.config1()[1]
    nb = C.c_size_t()
    assert L.hjm_workspace_bytes(hjm.make_axes(s.axes), s.n_steps, C.byref(nb)) == 0
    pts = 32 ** 3
    per_step = (2 * 32 + 32) * 8 * s.n_steps  # Dirichlet increments
    assert 3 * pts * 8 <= nb.value <= 3 * pts * 8 + per_step + 64 * 1024
    s3 = W.config3()[-1]
    assert L.hjm_workspace_bytes(hjm.make_axes(s3.axes), s3.n_steps, C.byref(nb)) == 0
    assert nb.value >= 3 * 256 * 128 * 128 * 8
    assert L.hjm_workspace_bytes(hjm.make_axes(s.axes), 0, C.byref(nb)) == hjm.EINVAL


def _bad_specs():
    s = W.config1()[1]
    ax = s.axes
    yield "n<5", replace(s, axes=(replace(ax[0], n=4), ax[1], ax[2]))
    yield "n too large", replace(s, axes=(replace(ax[0], n=5000), ax[1], ax[2]))
    yield "alpha<=0", replace(s, axes=(ax[0], replace(ax[1], alpha=0.0), ax[2]))
    yield "zmin>=zmax", replace(s, axes=(ax[0], ax[1], replace(ax[2], z_max=0.0)))
    yield "v dirichlet", replace(s, axes=(ax[0], replace(ax[1], lo_face=W.DIRICHLET), ax[2]))
    yield "y_lo dirichlet", replace(s, axes=(ax[0], ax[1], replace(ax[2], lo_face=W.DIRICHLET)))
    yield "face type", replace(s, axes=(replace(ax[0], hi_face=7), ax[1], ax[2]))
    yield "rho", replace(s, model=replace(s.model, rho=1.5))
    yield "eps<0", replace(s, model=replace(s.model, epsilon=-0.1))
    yield "kappa<0", replace(s, model=replace(s.model, kappa=-0.1))
    yield "gamma>1", replace(s, model=replace(s.model, gamma=1.2))
    yield "gamma>0 with r<0", replace(s, axes=(replace(ax[0], z_min=-0.1), ax[1], ax[2]))
    yield "nan", replace(s, model=replace(s.model, f_level=float("nan")))
    yield "expiry", replace(s, payoff=replace(s.payoff, expiry=0.0))
    yield "pay<=expiry", replace(s, payoff=replace(s.payoff, pay=1.0))
    yield "strike", replace(s, payoff=replace(s.payoff, strike=0.0))
    yield "kind", replace(s, payoff=replace(s.payoff, kind=9))
    yield "steps", replace(s, n_steps=0)
    # inflow at an outflow face: a falling curve makes f_t + kappa f < 0 at r = 0
    yield "r_min inflow", replace(s, model=replace(s.model, kappa=0.0, f_slope=-0.02, f_decay=1.0))
    yield "v_max inflow", replace(s, axes=(ax[0], replace(ax[1], z_max=0.9), ax[2]))
    yield "y_max outflow inflow", replace(s, axes=(ax[0], ax[1], replace(ax[2], hi_face=W.OUTFLOW)))


@pytest.mark.parametrize("name,spec", list(_bad_specs()))
def test_invalid_problems_rejected_on_host(L, name, spec):
    st, msg = _create(spec)
    assert st == hjm.EINVAL, (name, st, msg)
    assert msg


def test_workspace_too_small_and_misaligned(L):
    s = W.config1()[1]
    st, msg = _create(s, ws_bytes=1024)
    assert st == hjm.ENOMEM and "needs" in msg
    st, _ = _create(s, ws_ptr=0x100008)
    assert st == hjm.EINVAL
    st, _ = _create(s, ws_ptr=0)
    assert st == hjm.EINVAL


def test_null_handles(L):
    assert L.hjm_adi_step(None, 1) == hjm.EINVAL
    assert L.hjm_price(None, 0.03, 1.0, C.byref(C.c_double())) == hjm.EINVAL
    assert L.hjm_batch_run(None, 0) == hjm.EINVAL
    assert L.hjm_grid_plan(None, (C.c_int32 * 10)()) == hjm.EINVAL
    assert L.hjm_grid_profile_read(None, (C.c_double * hjm.N_PASSES)(), (C.c_int64 * hjm.N_PASSES)()) == hjm.EINVAL
    assert L.hjm_grid_destroy(None) == hjm.OK
    b = hjm.MlpBaseline(0.15, 0.9, 0.25, 0.5, 1.0)
    assert L.hjm_mlp_set_baseline(None, C.byref(b)) == hjm.EINVAL
    assert L.hjm_mlp_targets(None, None, None, 1, None) == hjm.EINVAL


def test_pass_count_matches_header():
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "hjm.h")).read()
    assert int(re.search(r"#define HJM_N_PASSES (\d+)", hdr).group(1)) == hjm.N_PASSES == len(hjm.PASSES)


def test_line_tile_setting(L):
    old = hjm.get_line_tile()
    try:
        hjm.set_line_tile(8, 32, 16)
        assert hjm.get_line_tile() == (8, 32, 16)
        with pytest.raises(hjm.HjmError):
            hjm.set_line_tile(12, 16, 16)
    finally:
        hjm.set_line_tile(*old)


def test_scheme_workspace_and_validation(L):
    """A correction scheme needs one more grid-sized array; unknown schemes,
    theta outside (0, 1] and grids without the lane-split r solve are
    rejected on the host."""
    from dataclasses import replace
    s = W.config1()[1]
    ax = hjm.make_axes(s.axes)
    dbl = hjm.workspace_bytes(s)
    cs = hjm.workspace_bytes(replace(s, scheme=W.CS))
    assert cs - dbl >= s.points * 8 and cs - dbl < s.points * 8 + 512
    nb = C.c_size_t()
    for kind, iters, theta in ((5, 0, 0.5), (-1, 0, 0.5), (W.CS, 0, 0.0), (W.MCS, 0, 1.5), (W.HV, 0, float("nan")),
                               (W.HUANG, 0, 0.5), (W.HUANG, 17, 0.5), (W.HUANG, -2, 0.5)):
        st = L.hjm_scheme_workspace_bytes(ax, 10, C.byref(hjm.Scheme(kind, iters, theta)), C.byref(nb))
        assert st == hjm.EINVAL, (kind, iters, theta)
    # Huang's correction reuses the correction array: the same workspace at any af_iters
    for q in (1, 16):
        assert hjm.workspace_bytes(replace(s, scheme=W.HUANG, af_iters=q)) == cs
    # nr = 40 has no power-of-two lane split: rejected before the workspace is touched
    bad = replace(W.with_shape(s, 40, 24, 32, 10), scheme=W.CS)
    h = C.c_void_p()
    st = L.hjm_grid_create_scheme(hjm.make_axes(bad.axes), C.byref(hjm.make_model(bad.model)),
                                  C.byref(hjm.make_payoff(bad.payoff)), C.byref(hjm.make_scheme(bad)), bad.n_steps,
                                  C.c_void_p(256), 1 << 40, None, C.byref(h))
    assert st == hjm.EINVAL and not h.value
    assert "lane-split" in L.hjm_last_error().decode()


def test_tuning_knobs(L):
    """Explicit chunk, r fusion and batch stream lanes: process-wide host
    settings, read back as set; invalid values rejected."""
    old_J, old_f = hjm.get_explicit_chunk(), hjm.get_r_fusion()
    try:
        for J in (4, 8, 16):
            hjm.set_explicit_chunk(J)
            assert hjm.get_explicit_chunk() == J
        with pytest.raises(hjm.HjmError):
            hjm.set_explicit_chunk(6)
        for on in (False, True):
            hjm.set_r_fusion(on)
            assert hjm.get_r_fusion() is on
        old_n = hjm.get_batch_streams()
        try:
            for n in (1, 3, 8):
                hjm.set_batch_streams(n)
                assert hjm.get_batch_streams() == n
            for bad in (0, 9):
                with pytest.raises(hjm.HjmError):
                    hjm.set_batch_streams(bad)
        finally:
            hjm.set_batch_streams(old_n)
        old_s = hjm.get_batch_share()
        try:
            for on in (False, True):
                hjm.set_batch_share(on)
                assert hjm.get_batch_share() is on
        finally:
            hjm.set_batch_share(old_s)
    finally:
        hjm.set_explicit_chunk(old_J)
        hjm.set_r_fusion(old_f)


def test_batch_validation(L):
    specs = W.config4(n=4)
    n = len(specs)
    ax = (hjm.Axis * (3 * n))()
    for s, sp in enumerate(specs):
        for a in range(3):
            ax[3 * s + a] = hjm.make_axes(sp.axes)[a]
    steps = (C.c_int32 * n)(*[sp.n_steps for sp in specs])
    nb = C.c_size_t()
    assert L.hjm_batch_workspace_bytes(n, ax, steps, C.byref(nb)) == 0
    assert nb.value >= sum(2 * sp.points * 8 for sp in specs)
    models = (hjm.Model * n)(*[hjm.make_model(sp.model) for sp in specs])
    pays = (hjm.Payoff * n)(*[hjm.make_payoff(sp.payoff) for sp in specs])
    pays[2].strike = -1.0
    h = C.c_void_p()
    st = L.hjm_batch_create(n, ax, models, pays, steps, C.c_void_p(0x100000), nb.value, None, C.byref(h))
    assert st == hjm.EINVAL and "solve 2" in L.hjm_last_error().decode()
    pays[2].strike = 0.03
    st = L.hjm_batch_create(n, ax, models, pays, steps, C.c_void_p(0x100000), 100, None, C.byref(h))
    assert st == hjm.ENOMEM


def test_discrete_curve_validation(L):
    """Discrete curves are checked on the host before any device work: knot
    count, the (0, 1) first knot, increasing maturities, positive finite
    prices."""
    from dataclasses import replace
    s = W.config_discrete((24, 12, 12))[0]
    ct, cp = list(s.model.curve_t), list(s.model.curve_p)
    bad = [(ct[:1], cp[:1]),                                   # one knot
           ([0.1] + ct[1:], cp),                               # first maturity not 0
           (ct, [0.99] + cp[1:]),                              # first price not 1
           (ct[:3] + [ct[2]] + ct[4:], cp),                    # maturities not increasing
           (ct, cp[:5] + [0.0] + cp[6:]),                      # price 0
           (ct, cp[:5] + [float("nan")] + cp[6:]),             # not finite
           ([i * 0.5 for i in range(65)], [1.0] + [0.99] * 64)]  # too many knots
    for t, p in bad:
        sp = replace(s, model=replace(s.model, curve_t=tuple(t), curve_p=tuple(p)))
        h = C.c_void_p()
        st = L.hjm_grid_create_scheme(hjm.make_axes(sp.axes), C.byref(hjm.make_model(sp.model)),
                                      C.byref(hjm.make_payoff(sp.payoff)), C.byref(hjm.make_scheme(sp)), sp.n_steps,
                                      C.c_void_p(256), 1 << 40, None, C.byref(h))
        assert st == hjm.EINVAL and not h.value, (t[:4], p[:6])
    m = hjm.make_model(s.model)
    m.curve_t = None
    h = C.c_void_p()
    st = L.hjm_grid_create_scheme(hjm.make_axes(s.axes), C.byref(m), C.byref(hjm.make_payoff(s.payoff)),
                                  C.byref(hjm.make_scheme(s)), s.n_steps, C.c_void_p(256), 1 << 40, None, C.byref(h))
    assert st == hjm.EINVAL and "null" in L.hjm_last_error().decode()


def test_hjm_run_argument_errors(tmp_path):
    """The command-line driver refuses bad arguments with its usage (exit 1)
    before it touches the device: no spec, an unknown option, and --graph
    without --batch (graph replay is a batch feature)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1108_1688_amd", "hjm_run")
    if not os.path.exists(exe):
        pytest.skip("hjm_run not built")
    spec = tmp_path / "one.spec"
    spec.write_text(W.spec_line(W.config1()[0]) + "\n")
    for args in ([], [str(spec), "--bogus"], [str(spec), "--graph"], [str(spec), "--batch", "--steps", "3"]):
        res = subprocess.run([exe, *args], capture_output=True, text=True, timeout=60)
        assert res.returncode == 1 and "usage: hjm_run" in res.stderr, (args, res.returncode, res.stderr)
