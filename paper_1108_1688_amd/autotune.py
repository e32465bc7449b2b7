"""Autotuner for the line-solve tiles and the explicit-kernel chunk.

The Douglas step is four kernels (explicit predictor, r, v and y sweeps) and
each one's speed depends on one setting only: the rows per thread of its own
line solve (r, v, y) or, for the explicit predictor, the v nodes per thread
(on grids whose r lines are solved inside the explicit kernel, the r rows).
The library times each kernel launch with HIP events, so a few runs along the
diagonal of the settings give every kernel's time for every candidate value,
and each kernel gets its own best value.

Timings are taken on representative solves (the largest by grid points times
steps) and weighted by the work each stands for; results are cached in a JSON
file keyed by the library build and the shapes, so a later process can reuse
them without timing again.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

from . import hjm

# (r rows, v rows, y rows, explicit chunk) along the diagonal: every kernel
# sees each of its candidate values once
DIAGONAL: Tuple[Tuple[int, int, int, int], ...] = ((8, 8, 8, 4), (16, 16, 16, 8), (32, 32, 32, 16))


@dataclass
class Tuning:
    setting: Tuple[int, int, int, int]        # (r, v, y, explicit chunk)
    per_pass_us: Dict[str, float]             # per Douglas step, for the chosen setting
    runs: List[dict] = field(default_factory=list)
    cached: bool = False

    def apply(self) -> None:
        r, v, y, J = self.setting
        hjm.set_line_tile(r, v, y)
        hjm.set_explicit_chunk(J)


def choose(runs: Sequence[dict], split: bool) -> Tuple[Tuple[int, int, int, int], Dict[str, float]]:
    """Pick each kernel's best value from diagonal runs.  A run is
    {"setting": (r, v, y, J), "us": [explicit, r, v, y]} with per-step
    microseconds (weighted over the representative solves).  When the r lines
    are solved inside the explicit kernel (split False), the explicit pass
    follows the r rows and the chunk is irrelevant."""
    def best(pass_idx, knob):
        run = min(runs, key=lambda x: x["us"][pass_idx])
        return run["setting"][knob], run["us"][pass_idx]

    if split:
        J, t0 = best(0, 3)
        r, t1 = best(1, 0)
    else:
        r, t0 = best(0, 0)
        J, t1 = hjm.get_explicit_chunk(), 0.0
    v, t2 = best(2, 1)
    y, t3 = best(3, 2)
    return (r, v, y, J), dict(zip(hjm.PASSES, (t0, t1, t2, t3)))


def _lib_id() -> str:
    with open(hjm.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _cache_key(specs: Sequence) -> str:
    shapes = sorted({(s.axes[0].n, s.axes[1].n, s.axes[2].n) for s in specs})
    return _lib_id() + ":" + ";".join("x".join(map(str, sh)) for sh in shapes)


def representatives(specs: Sequence, k: int = 3) -> List[Tuple[object, float]]:
    """Up to k solves of distinct shapes with the most work, each with the
    share of the total point-steps of its shape."""
    work: Dict[tuple, float] = {}
    pick: Dict[tuple, object] = {}
    for s in specs:
        sh = (s.axes[0].n, s.axes[1].n, s.axes[2].n)
        work[sh] = work.get(sh, 0.0) + s.points * s.n_steps
        if sh not in pick or s.n_steps > pick[sh].n_steps:
            pick[sh] = s
    top = sorted(work, key=work.get, reverse=True)[:k]
    total = sum(work.values())
    return [(pick[sh], work[sh] / total) for sh in top]


def tune(specs: Sequence, steps: int = 4, cache: Optional[str] = None, apply: bool = True) -> Tuning:
    """Time the diagonal settings on representative solves and choose each
    kernel's best value.  Restores the previous settings unless apply."""
    specs = list(specs)
    key = _cache_key(specs)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f).get(key)
        if stored:
            t = Tuning(tuple(stored["setting"]), stored["per_pass_us"], stored.get("runs", []), cached=True)
            if apply:
                t.apply()
            return t
    old_tile, old_J = hjm.get_line_tile(), hjm.get_explicit_chunk()
    reps = representatives(specs)
    runs = []
    split = True
    try:
        for setting in DIAGONAL:
            r, v, y, J = setting
            hjm.set_line_tile(r, v, y)
            hjm.set_explicit_chunk(J)
            us = [0.0] * hjm.N_PASSES
            for spec, weight in reps:
                n = min(steps + 1, spec.n_steps)
                g = hjm.Grid(spec)
                split = split and g.plan()["r_method"] == "split"
                g.step(1)  # warm-up
                g.profile(True)
                g.profile_read()
                g.step(n - 1)
                ms, cnt = g.profile_read()
                g.close()
                for q in range(hjm.N_PASSES):
                    if cnt[q]:
                        us[q] += weight * 1e3 * ms[q] / cnt[q]
            runs.append({"setting": setting, "us": us})
    finally:
        hjm.set_line_tile(*old_tile)
        hjm.set_explicit_chunk(old_J)
    setting, per_pass = choose(runs, split)
    result = Tuning(setting, per_pass, runs)
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key] = {"setting": list(setting), "per_pass_us": per_pass, "runs": runs}
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    if apply:
        result.apply()
    return result
