"""Launch-shape autotuner for the fused step kernels.

For a given grid (dimension, extents, dtype, batch, walls) it times the
candidate (variant, tile_rows) pairs -- one thread per cell, the marching
single-step kernels with several tile heights, and the multi-step passes of
2 to 8 levels with several wave heights, load groups and frame forms -- on the GPU
with HIP events, keeps the fastest, and caches the choice in a JSON file
keyed by the grid so later runs reuse it without timing.  ``tune_multi`` does
the same for a set of problems (single steps, or multi-step passes of 2 to 8
levels).
Every candidate computes the same result (the kernels evaluate the scheme in
the same operation order), so tuning never changes numerics.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

from . import (VARIANT_CELL, VARIANT_DEEP, VARIANT_FOURSTEP, VARIANT_MARCH, VARIANT_MARCH1, VARIANT_THREESTEP,
               VARIANT_TWOSTEP)

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")

# multi-step variants: rows per wave in the low 12 bits, load group size above
# (frame form in bits 16-19: spans of that many rows for the frame's steps as
# wave marches, 15 all of them fused in one launch; DEEP: levels per pass in
# bits 20-23, bit 24 loads issued a group ahead)
CANDIDATES_2D: List[Tuple[int, int]] = ([(VARIANT_DEEP, (pf << 24) | (d << 20) | (g << 12) | r)
                                         for d in (6, 8) for pf in (0, 1) for g in (2, 4) for r in (16, 24, 32, 48)]
                                        + [(VARIANT_DEEP, (pf << 24) | (7 << 20) | (2 << 12) | r)
                                           for pf in (0, 1) for r in (24, 32)]
                                        + [(VARIANT_DEEP, (d << 20) | (15 << 16) | (2 << 12) | 24) for d in (4, 6)]
                                        + [(VARIANT_FOURSTEP, (g << 12) | r) for g in (2, 4) for r in (8, 16)]
                                        + [(VARIANT_THREESTEP, (g << 12) | r) for g in (2, 4) for r in (6, 8, 12)]
                                        + [(VARIANT_THREESTEP, (f << 16) | (4 << 12) | 8) for f in (2, 3)]
                                        + [(VARIANT_TWOSTEP, (g << 12) | r) for g in (2, 4) for r in (8, 16)]
                                        + [(VARIANT_CELL, th) for th in (1, 2, 4, 8)]
                                        + [(VARIANT_MARCH, r) for r in (4, 8, 16)]
                                        + [(VARIANT_MARCH1, r) for r in (4, 8, 16)])
# 3D: marching single steps (k_march3d_plan: planes per core chunk in bits
# 0-11, rows per core wave in bits 12-15, rows per z/x-band wave in 16-17
# (0: 1, 1: 2, 2: 4), the core's waves first bit 18, planes per layer chunk
# in 20-27) and two-step passes (planes per chunk in bits 0-11, rows per wave
# in 12-17; bit 19 the marching frame with its layer chunk in 20-27; bit 28
# the core's tiles in launch order; bit 30 the frame as two levels per march
# with its shape in bits 18-29)
CANDIDATES_3D: List[Tuple[int, int]] = ([(VARIANT_CELL, 4)]
                                        + [(VARIANT_MARCH, (lc << 20) | (cf << 18) | (yl << 16) | (ry << 12) | ch)
                                           for ry, ch, lc, yl, cf in ((2, 16, 8, 0, 0), (4, 16, 8, 0, 0),
                                                                      (2, 16, 8, 1, 0), (2, 16, 8, 2, 0),
                                                                      (4, 16, 8, 2, 1), (2, 16, 8, 1, 1),
                                                                      (4, 32, 16, 2, 0))]
                                        + [(VARIANT_TWOSTEP, (ry << 12) | ch) for ry in (8, 16) for ch in (32, 64)]
                                        + [(VARIANT_TWOSTEP, (1 << 28) | (1 << 19) | (lc << 20) | (ry << 12) | ch)
                                           for ry, ch, lc in ((4, 64, 8), (8, 64, 8))]
                                        + [(VARIANT_TWOSTEP, (1 << 30) | (1 << 29) | (3 << 26) | (lc << 21) | (mc << 20)
                                            | (sm << 19) | (r4 << 18) | (ry << 12) | ch)
                                           for ry in (8, 16)
                                           for mc, sm, r4, lc, ch in ((1, 1, 1, 0, 32), (0, 1, 1, 0, 32), (1, 1, 0, 0, 32),
                                                                      (0, 0, 1, 0, 32), (1, 1, 1, 2, 64))])


def grid_key(sim) -> str:
    return "d%d_%s_N%s_b%d_w%s" % (sim.ndim, "f32" if sim.code == 0 else "f64",
                                   "x".join(str(n) for n in sim.N), sim.batch,
                                   "".join("1" if w else "0" for w in getattr(sim, "walls", ())) or "0")


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time_candidate(sim, variant: int, tile_rows: int, steps: int) -> float:
    torch = sim.torch
    sim.set_variant(variant, tile_rows)
    blob, n = sim.get_state()
    blob = blob.clone()
    sim.step(6)                                   # warm the code path (whole multi-step passes)
    sim.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    sim.put_state(blob, n)                       # leave the simulation where it was
    sim.sync()
    return e0.elapsed_time(e1) / steps


def tune(sim, steps: int = 50, candidates: Optional[Sequence[Tuple[int, int]]] = None,
         cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> Dict:
    """Pick and apply the fastest (variant, tile_rows) for ``sim`` (whose state
    must be set).  Returns {"variant", "tile_rows", "ms_per_step", "timings"}."""
    key = grid_key(sim)
    db = _load(cache) if cache else {}
    if not force and key in db:
        best = db[key]
        sim.set_variant(best["variant"], best["tile_rows"])
        return dict(best, cached=True)
    if candidates is None:
        candidates = CANDIDATES_2D if sim.ndim == 2 else CANDIDATES_3D
    timings = []
    for variant, rows in candidates:
        ms = _time_candidate(sim, variant, rows, steps)
        timings.append({"variant": variant, "tile_rows": rows, "ms_per_step": ms})
    best = min(timings, key=lambda t: t["ms_per_step"])
    rec = {"variant": best["variant"], "tile_rows": best["tile_rows"],
           "ms_per_step": best["ms_per_step"], "timings": timings}
    sim.set_variant(rec["variant"], rec["tile_rows"])
    if cache:
        db = _load(cache)
        db[key] = rec
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return dict(rec, cached=False)


# many-problem path: (variant, tile rows, rows loaded together)
CANDIDATES_MULTI: List[Tuple[int, int, int]] = ([(VARIANT_MARCH, r, g) for r in (8, 16, 32, 64) for g in (1, 2, 4)]
                                              + [(v, r, g) for v in (VARIANT_TWOSTEP, VARIANT_THREESTEP, VARIANT_FOURSTEP)
                                                 for r in (4, 8, 16) for g in (2, 4)]
                                              + [(VARIANT_DEEP, (d << 20) | r, g) for d in (5, 6, 8) for r in (8, 16, 32)
                                                 for g in (2, 4)])


def multi_key(multi) -> str:
    return "multi_%s_p%d_c%d_%s" % ("f32" if multi.code == 0 else "f64", multi.count, multi.cells,
                                    "-".join("x".join(str(n) for n in sh) for sh in multi.shapes[:4]))


def tune_multi(multi, U0s, steps: int = 20, candidates: Optional[Sequence[Tuple[int, int, int]]] = None,
               cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> Dict:
    """Pick and apply the fastest (variant, tile_rows, group) of the
    many-problem path for ``multi``, timing ``steps`` eager steps from
    ``U0s`` per candidate.  Leaves the problems at ``U0s``.  Returns
    {"variant", "tile_rows", "group", "ms_per_step", "timings"}."""
    torch = multi.torch
    key = multi_key(multi)
    db = _load(cache) if cache else {}
    if not force and key in db:
        best = db[key]
        multi.set_variant(best["variant"], best["tile_rows"], best["group"])
        multi.set_state(U0s)
        return dict(best, cached=True)
    timings = []
    for variant, rows, group in (candidates if candidates is not None else CANDIDATES_MULTI):
        multi.set_variant(variant, rows, group)
        multi.set_state(U0s)
        multi.step(2)
        multi.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        multi.step(steps)
        e1.record()
        torch.cuda.synchronize()
        timings.append({"variant": variant, "tile_rows": rows, "group": group,
                        "ms_per_step": e0.elapsed_time(e1) / steps})
    best = min(timings, key=lambda t: t["ms_per_step"])
    rec = {"variant": best["variant"], "tile_rows": best["tile_rows"], "group": best["group"],
           "ms_per_step": best["ms_per_step"], "timings": timings}
    multi.set_variant(rec["variant"], rec["tile_rows"], rec["group"])
    multi.set_state(U0s)
    if cache:
        db = _load(cache)
        db[key] = rec
        tmp = cache + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return dict(rec, cached=False)
