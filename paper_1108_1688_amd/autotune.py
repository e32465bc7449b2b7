"""Autotuner for the line-solve tiles, per line shape.

A Douglas step runs one kernel per direction (the explicit predictor fused
with the r sweep, then the v and y sweeps), and each kernel's speed depends
on the rows per thread of its own line solve and on the shape of its lines:
the line length n (the node count along its axis) and the number of lines
(the product of the other two node counts).  The library times each kernel
launch with HIP events, so timing every candidate value on every axis at
once (the settings (8, 8, 8), (16, 16, 16), (32, 32, 32)) gives each
kernel's time for each of its candidates on each grid shape; for every line
shape (axis, n, lines) the candidate with the least time, weighted by the
work (grid points times steps) of the solves that have that line shape,
wins.  The choices go to the library as per-shape overrides
(hjm_set_axis_tile), so that one batch runs each shape on its own best tiles.

Results are cached in a JSON file keyed by the device, the library build and
each line shape, so a later process reuses them without timing again.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

from . import hjm

CANDIDATES: Tuple[int, ...] = (8, 16, 32)
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
    choice: Dict[LineShape, int]                          # rows per thread of every line shape
    us: Dict[LineShape, Dict[int, float]]                 # weighted kernel time per candidate
    default_rows: Tuple[int, int, int] = (16, 16, 16)
    cached: bool = False
    timed_grids: int = 0

    def apply(self) -> None:
        """Install the choices as the library's per-shape overrides."""
        for (axis, n, lines), rows in self.choice.items():
            hjm.set_axis_tile(axis, n, lines, rows)

    def summary(self) -> dict:
        """Chosen rows per line shape ("r:96x9216" -> 16) and how many
        shapes differ from the default."""
        out = {f"{AXES[a]}:{n}x{lines}": rows for (a, n, lines), rows in sorted(self.choice.items())}
        differ = sum(1 for (a, _, _), rows in self.choice.items() if rows != self.default_rows[a])
        return {"per_line_shape": out, "line_shapes": len(self.choice), "differ_from_default": differ}


def choose(times: Dict[LineShape, Dict[int, float]]) -> Dict[LineShape, int]:
    """Each line shape's candidate with the least weighted time."""
    return {key: min(per, key=per.get) for key, per in times.items() if per}


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


def _key_str(dev: str, lib: str, key: LineShape) -> str:
    a, n, lines = key
    return f"{dev}:{lib}:{AXES[a]}:{n}:{lines}"


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


def time_shapes(shapes: Dict[tuple, Tuple[object, float]], steps: int) -> Dict[LineShape, Dict[int, float]]:
    """Per line shape and candidate: the weighted per-launch microseconds of
    that axis's kernel, from `steps` event-timed Douglas steps of one grid of
    every shape under each candidate setting (after one untimed step)."""
    times: Dict[LineShape, Dict[int, float]] = {}
    for rows in CANDIDATES:
        hjm.clear_axis_tiles()
        hjm.set_line_tile(rows, rows, rows)
        for sh, (spec, weight) in shapes.items():
            n = min(steps + 1, spec.n_steps)
            g = hjm.Grid(spec)
            g.step(1)
            g.profile(True)
            g.profile_read()
            g.step(n - 1)
            ms, cnt = g.profile_read()
            g.close()
            for key in line_shapes(sh):
                us = sum(1e3 * ms[q] / cnt[q] for q in PASS_OF_AXIS[key[0]] if cnt[q])
                times.setdefault(key, {})
                times[key][rows] = times[key].get(rows, 0.0) + weight * us
    return times


def tune(specs: Sequence, steps: int = 4, cache: Optional[str] = None, apply: bool = True) -> Tuning:
    """Choose the rows per thread of every line shape of specs (timing what
    the cache does not hold) and, if apply, install them as overrides; the
    global line tile is left as it was."""
    specs = list(specs)
    shapes = shapes_by_work(specs)
    keys = sorted({k for sh in shapes for k in line_shapes(sh)})
    dev, lib = _device_id(), _lib_id()
    old_tile = hjm.get_line_tile()
    stored = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
    if all(_key_str(dev, lib, k) in stored for k in keys):
        t = Tuning({k: stored[_key_str(dev, lib, k)]["rows"] for k in keys},
                   {k: {int(c): v for c, v in stored[_key_str(dev, lib, k)]["us"].items()} for k in keys},
                   old_tile, cached=True)
    else:
        try:
            times = time_shapes(shapes, steps)
        finally:
            hjm.clear_axis_tiles()
            hjm.set_line_tile(*old_tile)
        t = Tuning(choose(times), times, old_tile, timed_grids=len(shapes) * len(CANDIDATES))
        if cache:
            for k in keys:
                stored[_key_str(dev, lib, k)] = {"rows": t.choice[k], "us": {str(c): v for c, v in t.us[k].items()}}
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(stored, f, indent=1)
    if apply:
        t.apply()
    return t
