"""Thin ctypes binding of libhjm (include/hjm.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace tensors) and streams.
If libhjm.so has not been built this module raises on first use; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhjm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5
FACE_OUTFLOW, FACE_DIRICHLET = 0, 1
BOND, CAPLET, FLOORLET, FORWARD = 0, 1, 2, 3
N_PASSES = 4  # HJM_N_PASSES
PASSES = ("explicit", "r", "v", "y+update")
R_METHODS = ("spike", "chain", "split", "fused")
SCHEMES = ("douglas", "cs", "mcs", "hv", "huang")  # HJM_SCHEME_*
MLP_PARAMS = 199937  # HJM_MLP_PARAMS
STATIC_SCRATCH_BYTES = 32 << 20  # HJM_STATIC_SCRATCH_BYTES


class HjmError(RuntimeError):
    def __init__(self, status: int, text: str, detail: str):
        super().__init__(f"{text} ({detail})" if detail else text)
        self.status = status
        self.detail = detail


class Axis(C.Structure):
    _fields_ = [("n", C.c_int32), ("lo_face", C.c_int32), ("hi_face", C.c_int32), ("reserved", C.c_int32),
                ("z_min", C.c_double), ("z_max", C.c_double), ("center", C.c_double), ("alpha", C.c_double)]


class Model(C.Structure):
    _fields_ = [("kappa", C.c_double), ("theta_v", C.c_double), ("lam", C.c_double), ("gamma", C.c_double),
                ("epsilon", C.c_double), ("rho", C.c_double), ("f_level", C.c_double), ("f_slope", C.c_double),
                ("f_decay", C.c_double), ("curve_n", C.c_int32), ("reserved", C.c_int32),
                ("curve_t", C.POINTER(C.c_double)), ("curve_p", C.POINTER(C.c_double))]


class Payoff(C.Structure):
    _fields_ = [("kind", C.c_int32), ("soften", C.c_int32), ("expiry", C.c_double), ("pay", C.c_double),
                ("strike", C.c_double)]


class MlpBaseline(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("gamma", C.c_double), ("theta_v", C.c_double), ("f_decay", C.c_double),
                ("tenor", C.c_double)]


class Scheme(C.Structure):
    _fields_ = [("kind", C.c_int32), ("af_iters", C.c_int32), ("theta", C.c_double)]


_lib = None


def lib():
    """Load libhjm.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1108_1688_amd.build`")
    l = C.CDLL(LIB_PATH)
    st, vp, i32, i64, sz, d = C.c_int32, C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    P = C.POINTER
    sig = {
        "hjm_workspace_bytes": (st, [P(Axis), i32, P(sz)]),
        "hjm_grid_create": (st, [P(Axis), P(Model), P(Payoff), i32, vp, sz, vp, P(vp)]),
        "hjm_scheme_workspace_bytes": (st, [P(Axis), i32, P(Scheme), P(sz)]),
        "hjm_grid_create_scheme": (st, [P(Axis), P(Model), P(Payoff), P(Scheme), i32, vp, sz, vp, P(vp)]),
        "hjm_adi_step": (st, [vp, i32]),
        "hjm_price": (st, [vp, d, d, P(d)]),
        "hjm_grid_solution": (st, [vp, P(vp), P(i64)]),
        "hjm_grid_set_step": (st, [vp, i64]),
        "hjm_grid_destroy": (st, [vp]),
        "hjm_grid_plan": (st, [vp, P(i32)]),
        "hjm_grid_profile": (st, [vp, i32]),
        "hjm_grid_profile_read": (st, [vp, P(d), P(i64)]),
        "hjm_static_scratch_bytes": (st, [P(Axis), i32, P(sz)]),
        "hjm_price_static": (st, [P(Axis), P(Model), P(Payoff), i32, d, d, vp, vp, P(d)]),
        "hjm_batch_workspace_bytes": (st, [i32, P(Axis), P(i32), P(sz)]),
        "hjm_batch_create": (st, [i32, P(Axis), P(Model), P(Payoff), P(i32), vp, sz, vp, P(vp)]),
        "hjm_batch_scheme_workspace_bytes": (st, [i32, P(Axis), P(i32), P(Scheme), P(sz)]),
        "hjm_batch_create_scheme": (st, [i32, P(Axis), P(Model), P(Payoff), P(Scheme), P(i32), vp, sz, vp, P(vp)]),
        "hjm_batch_run": (st, [vp, i32]),
        "hjm_batch_prices": (st, [vp, P(d), P(d), P(d)]),
        "hjm_batch_greeks": (st, [vp, P(d), P(d), P(d)]),
        "hjm_price_greeks": (st, [vp, d, d, P(d)]),
        "hjm_batch_destroy": (st, [vp]),
        "hjm_batch_profile": (st, [vp, i32]),
        "hjm_batch_profile_read": (st, [vp, P(d), P(i64), P(i64)]),
        "hjm_set_line_tile": (st, [i32, i32, i32]),
        "hjm_get_line_tile": (st, [P(i32), P(i32), P(i32)]),
        "hjm_set_axis_tile": (st, [i32, i32, i64, i32]),
        "hjm_get_axis_tile": (st, [i32, i32, i64, P(i32)]),
        "hjm_clear_axis_tiles": (st, []),
        "hjm_set_explicit_chunk": (st, [i32]),
        "hjm_get_explicit_chunk": (st, [P(i32)]),
        "hjm_set_r_fusion": (st, [i32]),
        "hjm_get_r_fusion": (st, [P(i32)]),
        "hjm_set_exr_window": (st, [i32]),
        "hjm_get_exr_window": (st, [P(i32)]),
        "hjm_set_y_minors": (st, [i32]),
        "hjm_get_y_minors": (st, [P(i32)]),
        "hjm_set_v_fold": (st, [i32]),
        "hjm_get_v_fold": (st, [P(i32)]),
        "hjm_set_batch_streams": (st, [i32]),
        "hjm_get_batch_streams": (st, [P(i32)]),
        "hjm_set_batch_share": (st, [i32]),
        "hjm_get_batch_share": (st, [P(i32)]),
        "hjm_batch_operators": (st, [vp, P(i32)]),
        "hjm_mlp_workspace_bytes": (st, [i64, P(sz)]),
        "hjm_mlp_create": (st, [P(C.c_float), P(C.c_float), C.c_float, C.c_float, i64, vp, sz, vp, P(vp)]),
        "hjm_mlp_set_params": (st, [vp, P(C.c_float), i64]),
        "hjm_mlp_get_params": (st, [vp, P(C.c_float), i64]),
        "hjm_mlp_gradients": (st, [vp, vp, vp, i64, P(d)]),
        "hjm_mlp_get_grads": (st, [vp, P(C.c_float), i64]),
        "hjm_mlp_adam": (st, [vp, C.c_float, C.c_float, C.c_float, C.c_float]),
        "hjm_mlp_train_epoch": (st, [vp, vp, vp, i64, i64, C.c_float, P(d)]),
        "hjm_mlp_infer": (st, [vp, vp, i64, vp, vp]),
        "hjm_mlp_set_baseline": (st, [vp, vp]),
        "hjm_mlp_targets": (st, [vp, vp, vp, i64, vp]),
        "hjm_mlp_destroy": (st, [vp]),
        "hjm_status_str": (C.c_char_p, [st]),
        "hjm_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(l, name)
        fn.restype = res
        fn.argtypes = args
    _lib = l
    return l


def check(status: int) -> None:
    if status != OK:
        L = lib()
        raise HjmError(status, L.hjm_status_str(status).decode(), L.hjm_last_error().decode())


def make_axes(spec_axes) -> "C.Array":
    arr = (Axis * 3)()
    for a, s in zip(arr, spec_axes):
        a.n, a.lo_face, a.hi_face = s.n, s.lo_face, s.hi_face
        a.z_min, a.z_max, a.center, a.alpha = s.z_min, s.z_max, s.center, s.alpha
    return arr


def make_model(m) -> Model:
    """The model struct; a discrete curve (curve_t, curve_p) is copied into
    arrays that the returned struct keeps alive (the library reads them once,
    in the create call)."""
    mod = Model(m.kappa, m.theta_v, m.lam, m.gamma, m.epsilon, m.rho, m.f_level, m.f_slope, m.f_decay)
    ct, cp = getattr(m, "curve_t", None), getattr(m, "curve_p", None)
    if ct is not None:
        if cp is None or len(cp) != len(ct):
            raise ValueError("curve_t and curve_p must have the same length")
        t = (C.c_double * len(ct))(*[float(x) for x in ct])
        p = (C.c_double * len(cp))(*[float(x) for x in cp])
        mod.curve_n = len(ct)
        mod.curve_t = C.cast(t, C.POINTER(C.c_double))
        mod.curve_p = C.cast(p, C.POINTER(C.c_double))
        mod._knots = (t, p)
    return mod


def make_payoff(p) -> Payoff:
    return Payoff(p.kind, int(getattr(p, "soften", 0)), p.expiry, p.pay, p.strike)


def set_line_tile(r_rows: int, v_rows: int, y_rows: int) -> None:
    """Rows per thread of the r, v, y line solves (8, 16 or 32) for handles created afterwards."""
    check(lib().hjm_set_line_tile(r_rows, v_rows, y_rows))


def get_line_tile():
    r, v, y = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().hjm_get_line_tile(C.byref(r), C.byref(v), C.byref(y)))
    return r.value, v.value, y.value


def set_axis_tile(axis: int, n: int, lines: int, rows: int) -> None:
    """Preferred rows per thread (8, 16, 32; 0 clears) of the line solves
    along axis (0 r, 1 v, 2 y) on grids with n nodes there and `lines` such
    lines (0: any count), for handles created afterwards (overrides
    set_line_tile for that shape)."""
    check(lib().hjm_set_axis_tile(int(axis), int(n), int(lines), int(rows)))


def get_axis_tile(axis: int, n: int, lines: int = 0) -> int:
    r = C.c_int32()
    check(lib().hjm_get_axis_tile(int(axis), int(n), int(lines), C.byref(r)))
    return r.value


def clear_axis_tiles() -> None:
    check(lib().hjm_clear_axis_tiles())


def set_explicit_chunk(J: int) -> None:
    """v nodes per thread of the explicit-predictor kernel (4, 8 or 16) for handles created afterwards."""
    check(lib().hjm_set_explicit_chunk(J))


def get_explicit_chunk() -> int:
    J = C.c_int32()
    check(lib().hjm_get_explicit_chunk(C.byref(J)))
    return J.value


def set_r_fusion(on: bool) -> None:
    """Fuse the explicit predictor with the spike r solve where possible
    (default) or keep them as two kernels, for handles created afterwards."""
    check(lib().hjm_set_r_fusion(1 if on else 0))


def get_r_fusion() -> bool:
    on = C.c_int32()
    check(lib().hjm_get_r_fusion(C.byref(on)))
    return bool(on.value)


def set_exr_window(on: bool) -> None:
    """Explicit phase of the fused kernel from an LDS window (default) or
    from per-thread neighbour loads, for handles created afterwards."""
    check(lib().hjm_set_exr_window(1 if on else 0))


def get_exr_window() -> bool:
    on = C.c_int32()
    check(lib().hjm_get_exr_window(C.byref(on)))
    return bool(on.value)


def set_y_minors(on: bool) -> None:
    """y pivots formed in the y sweep each step from the minors recurrence
    (default) or stored once per solve, for handles created afterwards."""
    check(lib().hjm_set_y_minors(1 if on else 0))


def get_y_minors() -> bool:
    on = C.c_int32()
    check(lib().hjm_get_y_minors(C.byref(on)))
    return bool(on.value)


def set_v_fold(on: bool) -> None:
    """Douglas solves created afterwards fold the v sweep into the other
    kernels where they can (default), or run it on its own."""
    check(lib().hjm_set_v_fold(1 if on else 0))


def get_v_fold() -> bool:
    on = C.c_int32()
    check(lib().hjm_get_v_fold(C.byref(on)))
    return bool(on.value)


def set_batch_streams(n: int) -> None:
    """Stream lanes of batches created afterwards (1..8)."""
    check(lib().hjm_set_batch_streams(int(n)))


def get_batch_streams() -> int:
    n = C.c_int32()
    check(lib().hjm_get_batch_streams(C.byref(n)))
    return n.value


def set_batch_share(on: bool) -> None:
    """Whether batches created afterwards let solves of one operator (the
    right-hand sides: payoffs on the same mesh, model, dates and steps)
    share coefficient tables and y pivots."""
    check(lib().hjm_set_batch_share(1 if on else 0))


def get_batch_share() -> bool:
    n = C.c_int32()
    check(lib().hjm_get_batch_share(C.byref(n)))
    return bool(n.value)


def _torch():
    import torch
    return torch


def _workspace(nbytes: int, device):
    torch = _torch()
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace tensor is not 256-byte aligned")
    return ws


def make_scheme(spec) -> "Scheme":
    """The spec's ADI scheme (Douglas with theta = 1/2 unless it says otherwise)."""
    return Scheme(int(getattr(spec, "scheme", 0)), int(getattr(spec, "af_iters", 0)), float(getattr(spec, "theta", 0.5)))


def workspace_bytes(spec) -> int:
    nbytes = C.c_size_t()
    check(lib().hjm_scheme_workspace_bytes(make_axes(spec.axes), spec.n_steps, C.byref(make_scheme(spec)),
                                           C.byref(nbytes)))
    return nbytes.value


def _stream_handle(stream) -> C.c_void_p:
    return C.c_void_p(stream.cuda_stream if stream is not None else 0)


class Grid:
    """One solve: workspace in a torch tensor, work on a torch stream."""

    def __init__(self, spec, stream=None, device: Optional[str] = None, workspace=None):
        torch = _torch()
        L = lib()
        self.spec = spec
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ax = make_axes(spec.axes)
        self._model = make_model(spec.model)
        self._payoff = make_payoff(spec.payoff)
        self._scheme = make_scheme(spec)
        nbytes = C.c_size_t()
        check(L.hjm_scheme_workspace_bytes(self._ax, spec.n_steps, C.byref(self._scheme), C.byref(nbytes)))
        if workspace is not None:
            if workspace.dtype != torch.float64 or workspace.numel() * 8 < nbytes.value:
                raise ValueError("workspace must be a float64 tensor of at least the required bytes")
            if workspace.data_ptr() % 256:
                raise ValueError("workspace must be 256-byte aligned")
            self.ws = workspace
        else:
            self.ws = _workspace(nbytes.value, self.device)
        h = C.c_void_p()
        check(L.hjm_grid_create_scheme(self._ax, C.byref(self._model), C.byref(self._payoff),
                                       C.byref(self._scheme), spec.n_steps, C.c_void_p(self.ws.data_ptr()),
                                       nbytes.value, _stream_handle(self.stream), C.byref(h)))
        self._h = h

    def step(self, k: Optional[int] = None) -> "Grid":
        """Enqueue k Douglas steps (all remaining ones by default)."""
        if k is None:
            k = self.spec.n_steps - self.steps_taken
        check(lib().hjm_adi_step(self._h, int(k)))
        return self

    def price(self, r0: Optional[float] = None, v0: Optional[float] = None) -> float:
        out = C.c_double()
        r0 = self.spec.r0 if r0 is None else r0
        v0 = self.spec.v0 if v0 is None else v0
        check(lib().hjm_price(self._h, float(r0), float(v0), C.byref(out)))
        return out.value

    def greeks(self, r0: Optional[float] = None, v0: Optional[float] = None):
        """(price, rho = dC/dr, vega = dC/dv) at (r0, v0, y = 0)."""
        out = (C.c_double * 3)()
        r0 = self.spec.r0 if r0 is None else r0
        v0 = self.spec.v0 if v0 is None else v0
        check(lib().hjm_price_greeks(self._h, float(r0), float(v0), out))
        return tuple(out)

    @property
    def steps_taken(self) -> int:
        p, s = C.c_void_p(), C.c_int64()
        check(lib().hjm_grid_solution(self._h, C.byref(p), C.byref(s)))
        return s.value

    def solution(self):
        """The device grid U as a (ny, nv, nr) float64 view into the workspace."""
        p, s = C.c_void_p(), C.c_int64()
        check(lib().hjm_grid_solution(self._h, C.byref(p), C.byref(s)))
        off = (p.value - self.ws.data_ptr()) // 8
        npts = self.spec.points
        return self.ws[off:off + npts].view(*self.spec.shape)

    def set_step(self, step: int) -> None:
        check(lib().hjm_grid_set_step(self._h, int(step)))

    def plan(self) -> dict:
        """How this grid is solved: r method ('spike', 'chain', 'split' or
        'fused'), rows per lane of the split or fused r solve, line-tile rows, rows per segment
        of the segmented v solve and of the stored-pivot y solve (0 where the
        chained per-line solves are used instead), whether the y sweep forms
        its pivots from the minors recurrence and whether the v sweep is
        folded into the other kernels."""
        out = (C.c_int32 * 10)()
        check(lib().hjm_grid_plan(self._h, out))
        return {"r_method": R_METHODS[out[0]], "rs_rows": out[1], "line_tile": (out[2], out[3], out[4]),
                "vs_rows": out[5], "yc_rows": out[6], "scheme": SCHEMES[out[7]],
                "y_minors": bool(out[8]), "v_fold": bool(out[9])}

    def profile(self, enable: bool = True) -> None:
        """Bracket every pass launch with HIP events on the grid's stream."""
        check(lib().hjm_grid_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(ms per pass, launches per pass) since the last read; passes are
        PASSES (explicit, r, v, y+update; on grids that solve the r lines in the
        explicit kernel, pass 0 is both and pass 1 has no launches).
        Synchronises the stream."""
        ms = (C.c_double * N_PASSES)()
        n = (C.c_int64 * N_PASSES)()
        check(lib().hjm_grid_profile_read(self._h, ms, n))
        return list(ms), list(n)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().hjm_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def static_scratch_bytes(spec) -> int:
    """Bytes of the library's static device array that price_static needs for this solve."""
    nbytes = C.c_size_t()
    check(lib().hjm_static_scratch_bytes(make_axes(spec.axes), spec.n_steps, C.byref(nbytes)))
    return nbytes.value


def price_static(spec, U, stream=None, r0: Optional[float] = None, v0: Optional[float] = None):
    """One whole Douglas solve through hjm_price_static (no allocation in the
    library: its working arrays live in a static device array).  U is the
    caller's float64 CUDA tensor of spec.points elements (256-byte aligned);
    on return it holds the solution at t = 0.  Returns (price, rho, vega)."""
    torch = _torch()
    if U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous() or U.numel() != spec.points:
        raise ValueError("U must be a contiguous float64 CUDA tensor of spec.points elements")
    if U.data_ptr() % 256:
        raise ValueError("U must be 256-byte aligned")
    stream = stream if stream is not None else torch.cuda.current_stream(U.device)
    r0 = spec.r0 if r0 is None else r0
    v0 = spec.v0 if v0 is None else v0
    model = make_model(spec.model)
    out = (C.c_double * 3)()
    check(lib().hjm_price_static(make_axes(spec.axes), C.byref(model), C.byref(make_payoff(spec.payoff)),
                                 spec.n_steps, float(r0), float(v0), C.c_void_p(U.data_ptr()),
                                 _stream_handle(stream), out))
    return tuple(out)


class Batch:
    """Many independent solves advanced together (one launch per pass, sweep
    sequence and step); each solve's ADI scheme comes from its spec, as for
    Grid."""

    def __init__(self, specs: Sequence, stream=None, device: Optional[str] = None):
        torch = _torch()
        L = lib()
        self.specs = list(specs)
        n = len(self.specs)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ax = (Axis * (3 * n))()
        for s, sp in enumerate(self.specs):
            for a in range(3):
                x, y = self._ax[3 * s + a], sp.axes[a]
                x.n, x.lo_face, x.hi_face = y.n, y.lo_face, y.hi_face
                x.z_min, x.z_max, x.center, x.alpha = y.z_min, y.z_max, y.center, y.alpha
        self._model_refs = [make_model(sp.model) for sp in self.specs]  # keeps discrete curves alive
        self._models = (Model * n)(*self._model_refs)
        self._payoffs = (Payoff * n)(*[make_payoff(sp.payoff) for sp in self.specs])
        self._steps = (C.c_int32 * n)(*[sp.n_steps for sp in self.specs])
        self._schemes = (Scheme * n)(*[make_scheme(sp) for sp in self.specs])
        nbytes = C.c_size_t()
        check(L.hjm_batch_scheme_workspace_bytes(n, self._ax, self._steps, self._schemes, C.byref(nbytes)))
        self.ws = _workspace(nbytes.value, self.device)
        h = C.c_void_p()
        check(L.hjm_batch_create_scheme(n, self._ax, self._models, self._payoffs, self._schemes, self._steps,
                                        C.c_void_p(self.ws.data_ptr()), nbytes.value, _stream_handle(self.stream),
                                        C.byref(h)))
        self._h = h

    def run(self, graph: bool = False) -> "Batch":
        check(lib().hjm_batch_run(self._h, 1 if graph else 0))
        return self

    def profile(self, steps: int) -> None:
        """Time every launch of the first `steps` Douglas steps of eager runs."""
        check(lib().hjm_batch_profile(self._h, int(steps)))

    def profile_read(self):
        """(ms, launches, grid points) per pass since the last read."""
        ms = (C.c_double * N_PASSES)()
        n = (C.c_int64 * N_PASSES)()
        pts = (C.c_int64 * N_PASSES)()
        check(lib().hjm_batch_profile_read(self._h, ms, n, pts))
        return list(ms), list(n), list(pts)

    def prices(self, r0=None, v0=None) -> np.ndarray:
        n = len(self.specs)
        r0 = np.array([sp.r0 for sp in self.specs] if r0 is None else r0, dtype=np.float64)
        v0 = np.array([sp.v0 for sp in self.specs] if v0 is None else v0, dtype=np.float64)
        out = np.empty(n)
        dp = C.POINTER(C.c_double)
        check(lib().hjm_batch_prices(self._h, r0.ctypes.data_as(dp), v0.ctypes.data_as(dp), out.ctypes.data_as(dp)))
        return out

    def operators(self) -> int:
        """Distinct operators among the batch's solves (its length when
        sharing is off)."""
        n = C.c_int32()
        check(lib().hjm_batch_operators(self._h, C.byref(n)))
        return n.value

    def greeks(self, r0=None, v0=None) -> np.ndarray:
        """(n, 3): price, rho = dC/dr and vega = dC/dv of every solve."""
        n = len(self.specs)
        r0 = np.array([sp.r0 for sp in self.specs] if r0 is None else r0, dtype=np.float64)
        v0 = np.array([sp.v0 for sp in self.specs] if v0 is None else v0, dtype=np.float64)
        out = np.empty((n, 3))
        dp = C.POINTER(C.c_double)
        check(lib().hjm_batch_greeks(self._h, r0.ctypes.data_as(dp), v0.ctypes.data_as(dp), out.ctypes.data_as(dp)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().hjm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The surrogate network: parameters, optimiser state and activations in a
    workspace tensor, work on a torch stream.  Inputs are float32 (n, 8)
    device tensors in physical units; targets are in network units."""

    def __init__(self, box_lo, box_hi, out_scale: float, out_shift: float = 0.0, max_batch: int = 65536,
                 stream=None, device: Optional[str] = None):
        torch = _torch()
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.box_lo = np.asarray(box_lo, dtype=np.float32)
        self.box_hi = np.asarray(box_hi, dtype=np.float32)
        self.out_scale, self.out_shift, self.max_batch = float(out_scale), float(out_shift), int(max_batch)
        nbytes = C.c_size_t()
        check(L.hjm_mlp_workspace_bytes(self.max_batch, C.byref(nbytes)))
        self.ws = _workspace(nbytes.value, self.device)
        fp = C.POINTER(C.c_float)
        h = C.c_void_p()
        check(L.hjm_mlp_create(self.box_lo.ctypes.data_as(fp), self.box_hi.ctypes.data_as(fp), self.out_scale,
                               self.out_shift, self.max_batch, C.c_void_p(self.ws.data_ptr()), nbytes.value,
                               _stream_handle(self.stream), C.byref(h)))
        self._h = h
        self.baseline = None

    @staticmethod
    def _f32(a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float32)
        return a, a.ctypes.data_as(C.POINTER(C.c_float))

    def set_params(self, params: np.ndarray) -> None:
        a, ptr = self._f32(params)
        check(lib().hjm_mlp_set_params(self._h, ptr, a.size))

    def params(self) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.float32)
        check(lib().hjm_mlp_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    @staticmethod
    def _dev(t, cols=None):
        torch = _torch()
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected a contiguous float32 CUDA tensor")
        if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
            raise ValueError(f"expected shape (n, {cols})")
        return C.c_void_p(t.data_ptr())

    def gradients(self, x, t) -> float:
        """Summed squared error; the gradient stays on the device (grads())."""
        sse = C.c_double()
        check(lib().hjm_mlp_gradients(self._h, self._dev(x, 8), self._dev(t), x.shape[0], C.byref(sse)))
        return sse.value

    def grads(self) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.float32)
        check(lib().hjm_mlp_get_grads(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        check(lib().hjm_mlp_adam(self._h, lr, beta1, beta2, eps))

    def train_epoch(self, x, t, batch: int, lr: float) -> float:
        loss = C.c_double()
        check(lib().hjm_mlp_train_epoch(self._h, self._dev(x, 8), self._dev(t), x.shape[0], batch, lr,
                                        C.byref(loss)))
        return loss.value

    def set_baseline(self, lam: float, gamma: float, theta_v: float, f_decay: float, tenor: float) -> None:
        """Gaussian caplet baseline of the output (hjm_mlp_set_baseline)."""
        b = MlpBaseline(lam, gamma, theta_v, f_decay, tenor)
        check(lib().hjm_mlp_set_baseline(self._h, C.byref(b)))
        self.baseline = (lam, gamma, theta_v, f_decay, tenor)

    def clear_baseline(self) -> None:
        check(lib().hjm_mlp_set_baseline(self._h, None))
        self.baseline = None

    def targets(self, x, price):
        """Training targets (float32 device tensor) of prices (float64 device
        tensor) at rows x, in network units (hjm_mlp_targets)."""
        torch = _torch()
        if price.dtype != torch.float64 or not price.is_cuda or not price.is_contiguous() or price.dim() != 1:
            raise ValueError("expected a contiguous 1-D float64 CUDA tensor of prices")
        n = x.shape[0]
        if price.shape[0] != n:
            raise ValueError("one price per row")
        t = torch.empty(n, dtype=torch.float32, device=x.device)
        check(lib().hjm_mlp_targets(self._h, self._dev(x, 8), C.c_void_p(price.data_ptr()), n,
                                    C.c_void_p(t.data_ptr())))
        return t

    def infer(self, x):
        """(prices, in_box) device tensors for the rows of x."""
        torch = _torch()
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        inb = torch.empty(n, dtype=torch.uint8, device=x.device)
        check(lib().hjm_mlp_infer(self._h, self._dev(x, 8), n, C.c_void_p(y.data_ptr()), C.c_void_p(inb.data_ptr())))
        return y, inb

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().hjm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
