"""Autotuner for the line-solve tiles of a batch.

A Douglas step runs one kernel per direction (the explicit predictor fused
with the r sweep, then the v and y sweeps), and each kernel's speed depends
on the rows per thread of its own line solve and on the shape of its lines:
the line length n (the node count along its axis) and the number of lines
(the product of the other two node counts).

Two stages:

1. Per-kernel timing.  The library times each kernel launch with HIP events,
   so timing every candidate value on every axis at once (the settings
   (8, 8, 8), (16, 16, 16), (32, 32, 32)) on one grid of every distinct grid
   shape gives each kernel's time for each candidate on each line shape,
   weighted by the work (grid points times steps) of the solves with that
   line shape.  From these come two proposals: per line shape its fastest
   candidate, and per axis the candidate fastest summed over the axis's line
   shapes (one value per axis keeps a batch's launch groups whole).
2. End-to-end check.  A batch launches one kernel per launch group, and
   solves whose rows differ fall into separate groups: more, smaller
   launches per step, which the per-kernel times do not see.  So each
   proposal, and the default (no overrides), prices the whole batch a few
   times; the fastest wins and goes to the library as per-shape overrides
   (hjm_set_axis_tile).  With those tiles the batch is then priced over
   the candidate stream-lane counts (LANES), and the fastest count is kept
   (hjm_set_batch_streams).

Results are cached in a JSON file: the per-kernel times under (device,
library build, axis, nodes per line, lines), reused by any later batch that
has that line shape, and the batch-level choice under (device, build, the
batch's workload), so a later process reuses them without timing again.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

from . import hjm

CANDIDATES: Tuple[int, ...] = (8, 16, 32)
LANES: Tuple[int, ...] = (2, 3, 4)
AXES = ("r", "v", "y")
# the pass of each axis's line solve in the per-pass timing (on grids whose
# r lines are solved inside the explicit kernel, pass 0 holds both)
PASS_OF_AXIS = {0: (0, 1), 1: (2,), 2: (3,)}

LineShape = Tuple[int, int, int]  # (axis, nodes per line, lines)


def line_shapes(shape: Tuple[int, int, int]) -> List[LineShape]:
    """The three line shapes of an nr x nv x ny grid."""
    nr, nv, ny = shape
    return [(0, nr, nv * ny), (1, nv, nr * ny), (2, ny, nr * nv)]


@dataclass
class Tuning:
    choice: Dict[LineShape, int]                          # overrides installed (empty: the default)
    us: Dict[LineShape, Dict[int, float]]                 # weighted kernel time per candidate
    default_rows: Tuple[int, int, int] = (16, 16, 16)
    cached: bool = False
    timed_grids: int = 0
    per_shape: Dict[LineShape, int] = field(default_factory=dict)   # proposal: fastest per line shape
    per_axis: Dict[LineShape, int] = field(default_factory=dict)    # proposal: one value per axis
    batch_ms: Dict[str, float] = field(default_factory=dict)        # whole-batch time of each proposal
    chosen: str = "default"
    lanes: int = 0                                                  # stream lanes chosen (0: left as it was)
    lanes_ms: Dict[int, float] = field(default_factory=dict)        # whole-batch time per lane count

    def apply(self) -> None:
        """Install the chosen overrides (and lane count) in the library."""
        for (axis, n, lines), rows in self.choice.items():
            hjm.set_axis_tile(axis, n, lines, rows)
        if self.lanes:
            hjm.set_batch_streams(self.lanes)

    def summary(self) -> dict:
        """The chosen proposal, its rows per line shape ("r:96x9216" -> 16),
        how many shapes differ from the default, and every proposal's batch
        time."""
        out = {f"{AXES[a]}:{n}x{lines}": rows for (a, n, lines), rows in sorted(self.choice.items())}
        differ = sum(1 for (a, _, _), rows in self.choice.items() if rows != self.default_rows[a])
        return {"chosen": self.chosen, "per_line_shape": out, "line_shapes": len(self.per_shape),
                "differ_from_default": differ, "batch_ms": {k: round(v, 3) for k, v in self.batch_ms.items()},
                "lanes": self.lanes, "lanes_ms": {str(k): round(v, 3) for k, v in self.lanes_ms.items()}}


def choose(times: Dict[LineShape, Dict[int, float]]) -> Dict[LineShape, int]:
    """Each line shape's candidate with the least weighted time."""
    return {key: min(per, key=per.get) for key, per in times.items() if per}


def choose_per_axis(times: Dict[LineShape, Dict[int, float]]) -> Dict[LineShape, int]:
    """One candidate per axis, the least weighted time summed over the axis's
    line shapes (candidates timed on every one of them), for every line shape
    of that axis."""
    best: Dict[int, int] = {}
    for axis in range(3):
        keys = [k for k in times if k[0] == axis]
        common = set(CANDIDATES)
        for k in keys:
            common &= set(times[k])
        if keys and common:
            best[axis] = min(sorted(common), key=lambda c: sum(times[k][c] for k in keys))
    return {k: best[k[0]] for k in times if k[0] in best}


def _device_id() -> str:
    try:
        import torch
        p = torch.cuda.get_device_properties(0)
        return getattr(p, "gcnArchName", p.name).split(":")[0]
    except Exception:
        return "unknown"


def _lib_id() -> str:
    with open(hjm.LIB_PATH, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def shapes_by_work(specs: Sequence) -> Dict[Tuple[int, int, int], Tuple[object, float]]:
    """Each distinct grid shape of specs: a solve of that shape (the one with
    the most steps) and the shape's share of all point-steps."""
    work: Dict[tuple, float] = {}
    pick: Dict[tuple, object] = {}
    for s in specs:
        sh = (s.axes[0].n, s.axes[1].n, s.axes[2].n)
        work[sh] = work.get(sh, 0.0) + s.points * s.n_steps
        if sh not in pick or s.n_steps > pick[sh].n_steps:
            pick[sh] = s
    total = sum(work.values())
    return {sh: (pick[sh], work[sh] / total) for sh in work}


def workload_key(specs: Sequence, tile: Tuple[int, int, int]) -> str:
    """A digest of what the tuning depends on: every grid shape's work and
    steps, and the global line tile the default runs on."""
    sig = sorted(((sh, round(w, 12), spec.n_steps) for sh, (spec, w) in shapes_by_work(specs).items()))
    return hashlib.sha256(json.dumps([sig, list(tile), len(specs)]).encode()).hexdigest()[:16]


def time_shapes(shapes: Dict[tuple, Tuple[object, float]], steps: int,
                known: Optional[Dict[LineShape, Dict[int, float]]] = None) -> Tuple[Dict[LineShape, Dict[int, float]], int]:
    """Per line shape and candidate: the per-launch microseconds of that
    axis's kernel, from `steps` event-timed Douglas steps of one grid of every
    shape under each candidate setting (after one untimed step).  Line shapes
    in `known` keep their times, and grid shapes whose three line shapes are
    all known are not run.  Returns the times and the grids timed."""
    raw: Dict[LineShape, Dict[int, float]] = {k: dict(v) for k, v in (known or {}).items()}
    todo = {sh: v for sh, v in shapes.items() if not all(k in raw for k in line_shapes(sh))}
    fresh: Dict[LineShape, Dict[int, List[float]]] = {}
    for rows in CANDIDATES:
        hjm.clear_axis_tiles()
        hjm.set_line_tile(rows, rows, rows)
        for sh, (spec, _) in todo.items():
            n = min(steps + 1, spec.n_steps)
            g = hjm.Grid(spec)
            g.step(1)
            g.profile(True)
            g.profile_read()
            g.step(n - 1)
            ms, cnt = g.profile_read()
            g.close()
            for key in line_shapes(sh):
                if key in raw:
                    continue
                us = sum(1e3 * ms[q] / cnt[q] for q in PASS_OF_AXIS[key[0]] if cnt[q])
                fresh.setdefault(key, {}).setdefault(rows, []).append(us)
    # a line shape met in several grid shapes: the mean of its measurements
    for key, per in fresh.items():
        raw[key] = {rows: sum(v) / len(v) for rows, v in per.items()}
    return raw, len(todo) * len(CANDIDATES)


def weigh(raw: Dict[LineShape, Dict[int, float]], shapes: Dict[tuple, Tuple[object, float]]) -> Dict[LineShape, Dict[int, float]]:
    """Each line shape's times weighted by the work share of the grid shapes
    that have it."""
    w: Dict[LineShape, float] = {}
    for sh, (_, weight) in shapes.items():
        for key in line_shapes(sh):
            w[key] = w.get(key, 0.0) + weight
    return {key: {rows: w[key] * us for rows, us in raw[key].items()} for key in w if key in raw}


def time_batch(specs: Sequence, overrides: Dict[LineShape, int], reps: int) -> float:
    """Milliseconds per priced run of the whole batch (eager launches on a
    stream of its own; one untimed run, then the median of reps) with the
    given overrides installed; the overrides are cleared afterwards."""
    import torch
    hjm.clear_axis_tiles()
    try:
        for (axis, n, lines), rows in overrides.items():
            hjm.set_axis_tile(axis, n, lines, rows)
        b = hjm.Batch(specs, stream=torch.cuda.Stream())
        try:
            b.run()
            b.prices()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                b.run()
                b.prices()
                ts.append(time.perf_counter() - t0)
        finally:
            b.close()
    finally:
        hjm.clear_axis_tiles()
    ts.sort()
    return 1e3 * ts[len(ts) // 2]


def tune(specs: Sequence, steps: int = 4, cache: Optional[str] = None, apply: bool = True,
         batch_reps: int = 3, lanes: bool = True) -> Tuning:
    """Choose the line tiles of the batch specs (timing what the cache does
    not hold) and, if lanes, the stream-lane count; if apply, install them
    (per-shape overrides, hjm_set_batch_streams).  The global line tile is
    left as it was; the lane count, if chosen, is process-wide."""
    specs = list(specs)
    shapes = shapes_by_work(specs)
    old_tile = tuple(hjm.get_line_tile())
    dev, lib = _device_id(), _lib_id()
    key = f"batch:{dev}:{lib}:{workload_key(specs, old_tile)}"
    stored = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)

    def line_key(k: LineShape) -> str:
        return f"line:{dev}:{lib}:{AXES[k[0]]}:{k[1]}:{k[2]}"

    def keys_of(d):
        return {tuple(int(x) for x in k.split(",")): v for k, v in d.items()}

    def str_keys(d):
        return {",".join(map(str, k)): v for k, v in d.items()}

    if key in stored and (stored[key]["lanes"] or not lanes):
        e = stored[key]
        raw = {k: {int(c): v for c, v in stored[line_key(k)]["us"].items()}
               for sh in shapes for k in line_shapes(sh) if line_key(k) in stored}
        t = Tuning(keys_of(e["choice"]), weigh(raw, shapes), old_tile, cached=True,
                   per_shape=keys_of(e["per_shape"]), per_axis=keys_of(e["per_axis"]),
                   batch_ms=e["batch_ms"], chosen=e["chosen"], lanes=e["lanes"] if lanes else 0,
                   lanes_ms={int(k): v for k, v in e["lanes_ms"].items()} if lanes else {})
    else:
        # per-kernel times: the cache's per line shape (device, build, axis,
        # nodes, lines), the rest measured
        known = {k: {int(c): v for c, v in stored[line_key(k)]["us"].items()}
                 for sh in shapes for k in line_shapes(sh) if line_key(k) in stored}
        try:
            raw, timed = time_shapes(shapes, steps, known)
        finally:
            hjm.clear_axis_tiles()
            hjm.set_line_tile(*old_tile)
        times = weigh(raw, shapes)
        proposals = {"default": {}, "per_axis": choose_per_axis(times), "per_shape": choose(times)}
        batch_ms = {name: time_batch(specs, ov, batch_reps) for name, ov in proposals.items()}
        chosen = min(batch_ms, key=batch_ms.get)
        t = Tuning(proposals[chosen], times, old_tile, timed_grids=timed,
                   per_shape=proposals["per_shape"], per_axis=proposals["per_axis"], batch_ms=batch_ms,
                   chosen=chosen)
        if lanes:
            old_lanes = hjm.get_batch_streams()
            try:
                for n in LANES:
                    hjm.set_batch_streams(n)
                    t.lanes_ms[n] = batch_ms[chosen] if n == old_lanes else time_batch(specs, t.choice, batch_reps)
            finally:
                hjm.set_batch_streams(old_lanes)
            t.lanes = min(t.lanes_ms, key=t.lanes_ms.get)
        if cache:
            for k, per in raw.items():
                stored[line_key(k)] = {"us": {str(c): v for c, v in per.items()}}
            stored[key] = {"choice": str_keys(t.choice), "per_shape": str_keys(t.per_shape),
                           "per_axis": str_keys(t.per_axis), "batch_ms": t.batch_ms, "chosen": t.chosen,
                           "lanes": t.lanes, "lanes_ms": {str(k): v for k, v in t.lanes_ms.items()}}
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(stored, f, indent=1)
    if apply:
        hjm.clear_axis_tiles()
        t.apply()
    return t
