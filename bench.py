"""Throughput benchmark of the fused discrete-PML step on one MI355X.

Headline workload: 3D, 512^3 interior + 24-cell layer on all six faces
(560^3 cells), FP64 (the precision of the paper's runs), c = 1, dt = 0.4 h,
damping ramping quadratically to 2/h, a Ricker point source at the centre
(15 points per wavelength) and the z plane through it recorded every step.
A step is one full pass of the method over the grid: U by leapfrog with the
layer terms, Phi_a and Psi_a of all three axes, the source and the plane.
The timed region is exactly --steps steps of the workload from rest (steps
0 .. K-1 of its 1000), launched as the tuned launch shape.

Prints ONE JSON line:
  value         Gcell-updates/s (all 560^3 cells per step, layer included)
  roofline      the dominant step kernel of the headline: its algorithmic
                bytes per launch (a single step: 3 words per cell + 4 per layer
                axis-cell; a multi-step pass's core: 4 words per core cell)
                over its mean launch duration (HIP events around each launch,
                on the stream it runs on) vs 8 TB/s, with the HBM bytes the
                rocprofv3 counters measured for that kernel when a summary for
                the current sources is committed under profiles/
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
  runs          the headline and the secondary single-grid records (3D FP32,
                the 2D 4160^2 workload in FP32 and FP64)

    python bench.py [--gpus 1] [--steps 1000] [--warmup 20]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gcell-updates/s incl. PML fields + % HBM peak; adjoint/forward time ratio"


def alg_bytes_per_step(w, esize: int) -> int:
    """3 words per cell (read U^n, read U^{n-1}, write U^{n+1}) + 4 words per
    layer axis-cell (read and write Phi_a, Psi_a); neighbour re-reads and the
    damping tables are not counted."""
    cells = w.cells
    aux = 0
    for a in range(w.ndim):
        M = w.lo[a] + w.hi[a]
        aux += M * (cells // w.N[a])
    return 3 * cells * esize + 4 * aux * esize


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_gpu(w, dtype_name, steps, warmup, variant=0, tile_rows=0):
    import torch
    import paper_1804_01390_amd as dp
    from paper_1804_01390_amd import autotune
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_state(torch.from_numpy(w.U0))
    if variant == 0:
        choice = autotune.tune(sim)           # cached per grid after the first run
        launch = {"variant": choice["variant"], "tile_rows": choice["tile_rows"],
                  "autotuned": True, "cached": choice["cached"]}
    else:
        sim.set_variant(variant, tile_rows)
        launch = {"variant": variant, "tile_rows": tile_rows, "autotuned": False}
    sim.set_state(torch.from_numpy(w.U0))
    sim.step(warmup)
    sim.sync()
    stream = torch.cuda.current_stream()
    # whole-job throughput: exactly `steps` steps between two synchronised
    # events, once with eager launches and once as one HIP-graph replay of
    # the whole run (captured and instantiated beforehand); the faster counts
    runs = {}
    for mode in ("eager", "graph"):
        sim.set_state(torch.from_numpy(w.U0))
        if mode == "graph":
            # capture + instantiate (+ one run) from the same rotation state the
            # timed replay starts from, so the timed call reuses the graph
            sim.step(warmup)
            sim.step_graph(steps)
            sim.set_state(torch.from_numpy(w.U0))
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        (sim.step_graph if mode == "graph" else sim.step)(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        runs[mode] = e0.elapsed_time(e1)
    total_ms = min(runs.values())
    # per-launch durations of the step kernels: the library brackets each
    # launch with a HIP event pair on its own stream (timing off above)
    k = min(steps, 200) // 2 * 2
    sim.set_timing(True)
    sim.step(k)
    kernels = sim.get_timing()
    sim.set_timing(False)
    ok = bool(np.isfinite(sim.U.float().abs().max().item()))
    sim.close()
    launch["timed"] = min(runs, key=runs.get)
    launch["eager_ms_per_step"] = round(runs["eager"] / steps, 5)
    launch["graph_ms_per_step"] = round(runs["graph"] / steps, 5)
    return {"total_ms": total_ms, "ms_per_step": total_ms / steps, "kernels": kernels, "timed_steps": k,
            "finite": ok, "launch": launch}


VALU_PEAK_WPS = 256 * 2.4e9          # wave64 VALU instructions per second over 256 CUs


def roofline_from_timing(kernels, timed_steps, workload=None, dtype_name=None):
    """Roofline of the dominant step kernel from the library's per-launch
    timing: its algorithmic bytes per launch over its mean launch duration.
    The dominant kernel is the class that moves the most algorithmic bytes:
    frame launches run on a second stream beside the core, so their event
    durations include time spent sharing the GPU and are no measure of which
    kernel carries the step.  With a committed counter summary for this
    workload, dtype and kernel class (and the current sources), ``traffic`` is
    the HBM bytes per launch it measured and ``hbm_GBps``/``hbm_frac`` that
    traffic over the same mean duration, and ``valu_frac`` its VALU wave
    instructions per launch over the same duration against the issue peak."""
    name, k = max(((n, v) for n, v in kernels.items() if v["launches"]), key=lambda kv: kv[1]["bytes"])
    ms = k["ms"] / k["launches"]
    bpl = k["bytes"] / k["launches"]
    achieved = bpl / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
           "alg_bytes_per_launch": int(round(bpl)), "kernel_ms_mean": round(ms, 5),
           "launches": k["launches"], "timed_steps": timed_steps}
    if workload:
        rec = traffic_from_profile(workload, dtype_name, name)
        if rec and rec.get("bytes_per_launch"):
            t = rec["bytes_per_launch"]
            out["traffic"] = int(t)
            out["hbm_GBps"] = round(t / (ms * 1e-3) / 1e9, 1)
            out["hbm_frac"] = round(t / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        if rec and rec.get("valu_wave_instr_per_launch"):
            # VALU issue: one wave64 instruction per cycle per CU (non-packed, no FMA)
            out["valu_frac"] = round(rec["valu_wave_instr_per_launch"] / (ms * 1e-3) / VALU_PEAK_WPS, 4)
    return out


def path_hbm(roof, kernels, timed_steps, ms_per_step, workload, dtype_name):
    """The whole path's HBM rate: the counter-measured bytes per launch of
    every kernel class in the timing run, summed over its launches, over the
    same number of steps at the measured time per step (classes run side by
    side on two streams, so durations do not add).  Needs a current counter
    record for every class."""
    total = 0.0
    for name, v in kernels.items():
        if not v["launches"]:
            continue
        rec = traffic_from_profile(workload, dtype_name, name)
        if not rec or not rec.get("bytes_per_launch"):
            return
        total += v["launches"] * rec["bytes_per_launch"]
    gbps = total / (timed_steps * ms_per_step * 1e-3) / 1e9
    roof["path_hbm_GBps"] = round(gbps, 1)
    roof["path_hbm_frac"] = round(gbps / HBM_PEAK_GBS, 4)


def cpu_baseline(w, sample_steps: int, U0=None):
    """The FP64 oracle on the same workload (its sources included) for
    `sample_steps` steps from rest."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    U0 = w.U0 if w.U0 is not None else np.zeros(tuple(reversed(w.N)))
    s = oracle.start(g, U0)
    kw = {}
    if w.sources:
        kw = {"sources": w.sources, "wavelets": w.wavelets, "nt": w.wavelets.shape[1]}
    # a run copies the state in and out of private buffers; the time of a
    # run of no steps (the same copies) is taken off a run of sample_steps
    oracle.run(g, s, 0, **kw)
    t = time.perf_counter()
    oracle.run(g, s, 0, **kw)
    t0 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.run(g, s, sample_steps, **kw)
    t1 = time.perf_counter() - t
    dt = t1 - t0
    shape = "x".join(str(n) for n in w.N)
    return {"value": round(sample_steps * w.cells / dt / 1e9, 5), "unit": "Gcell/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps (from rest, source included) of the same %s-cell workload, FP64, OpenMP over "
                      "cells; a %d-step run (%.1f s) minus a run of no steps (%.1f s: the state copies)"
                      % (sample_steps, shape, sample_steps, t1, t0),
            "seconds": round(dt, 3)}


def traffic_from_profile(workload: str, dtype_name: str, kernel: str):
    """The counter record of a step-kernel class (HBM bytes and VALU wave
    instructions per launch, measured by rocprofv3), if one for the current
    kernel sources is committed under profiles/."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (workload, dtype_name, kernel))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    import hashlib
    h = hashlib.sha256()
    for p in rec.get("sources", []):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None                # the kernel changed since the counters were taken
    return rec


def copy_probe(mib: int = 1024, reps: int = 20):
    """The library's streaming probe (read-only, write-only, copy; plain and
    non-temporal) over a buffer of known size: the bandwidth HBM gives a
    plain streaming kernel on this GPU, and the reference for scaling the
    rocprofv3 counters FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    import paper_1804_01390_amd as dp
    nb = mib << 20
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    src.random_(0, 255)
    dst = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = {"probe_bytes": nb}
    for kind, name in ((dp.PROBE_READ, "read"), (dp.PROBE_WRITE, "write"), (dp.PROBE_COPY, "copy")):
        for nt in (0, dp.PROBE_NONTEMPORAL):
            best = 0.0
            for bpc in (1, 2, 4, 8):
                dp.bandwidth_probe(kind | nt, nb, reps=2, blocks_per_cu=bpc, buffers=(dst, src))
                ms = dp.bandwidth_probe(kind | nt, nb, reps=reps, blocks_per_cu=bpc, buffers=(dst, src))
                gbs = nb * (2 if kind == dp.PROBE_COPY else 1) / (ms * 1e-3) / 1e9
                out["%s%s_b%d_GBps" % (name, "_nt" if nt else "", bpc)] = round(gbs, 1)
                best = max(best, gbs)
            out["%s%s_best_GBps" % (name, "_nt" if nt else "")] = round(best, 1)
    print(json.dumps(out), flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_ricker3d(steps: int, warmup: int, dtype_name: str = "f64", variant: int = 0, tile_rows: int = 0):
    """3D, 512^3 interior + 24-cell layer on all faces (560^3 cells),
    dt = 0.4 h, Ricker point source at the centre, the z plane through it
    recorded every step: `steps` steps of the workload from rest, after
    `warmup` untimed steps, in the tuned launch (or the given variant and
    launch shape)."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    from paper_1804_01390_amd import autotune
    w = synthetic.ricker3d(n=512, m=24, steps=1000)
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    esize = 4 if dtype_name == "f32" else 8
    if steps > w.steps:
        raise SystemExit("the 3D workload has %d steps" % w.steps)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    rest = lambda: torch.zeros(tuple(reversed(w.N)), dtype=dtype, device="cuda")
    sim.set_state(rest())
    sim.inject(w.sources, torch.from_numpy(w.wavelets).to(dtype))
    axis, index = w.plane
    sim.record_plane(axis, index, w.steps)
    if variant:
        sim.set_variant(variant, tile_rows)
        choice = {"variant": variant, "tile_rows": tile_rows, "cached": False}
    else:
        choice = autotune.tune(sim, steps=10)
    sim.set_state(rest())
    sim.step(warmup)
    sim.sync()
    # restart from rest so the timed run is the workload's steps 0 .. steps-1
    sim.set_state(rest())
    sim.sync()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    plane_cells = w.N[0] * w.N[1]
    ab = alg_bytes_per_step(w, esize) + plane_cells * esize
    peak = float(sim._keep["planes"][steps - 1].abs().max().item())
    # per-launch durations of the step kernels on a restarted run (library
    # events on each launch's stream; timing is off in the timed region)
    k = max(2, min(steps, 50) // 2 * 2)
    sim.set_state(rest())
    sim.set_timing(True)
    sim.step(k)
    kernels = sim.get_timing()
    sim.set_timing(False)
    roof = roofline_from_timing(kernels, k, "ricker3d_512_m24", dtype_name)
    roof["path_alg_GBps"] = round(ab * steps / (ms * 1e-3) / 1e9, 1)
    path_hbm(roof, kernels, k, ms / steps, "ricker3d_512_m24", dtype_name)
    sim.close()
    return {"dtype": dtype_name,
            "workload": "3D 512^3 interior + 24-cell layer on all six faces (560^3 cells), %s, c=1, dt=0.4h, "
                        "quadratic damping ramp to 2/h, Ricker point source at the centre (15 points per "
                        "wavelength), the z plane through it recorded every step; steps 0..%d of the workload's "
                        "%d timed after %d warmup steps" % (dtype_name.upper(), steps - 1, w.steps, warmup),
            "cells": w.cells, "steps": steps,
            "value": round(w.cells * steps / (ms * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "ms_per_step": round(ms / steps, 5),
            "alg_bytes_per_step": ab,
            "alg_GBps": round(ab * steps / (ms * 1e-3) / 1e9, 1),
            "plane_peak": peak, "roofline": roof, "kernels": kernels,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": not variant,
                       "cached": choice["cached"]}}


def bench_rk4(steps: int = 200):
    """The paper's own integrator (classic RK4 on U, V, Phi, Psi; four fused
    stage sweeps per step) on the 4160^2 FP32 workload, against leapfrog
    steps of the same grid."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    w = synthetic.bumps2d(n=4096, m=32, steps=steps, seed=0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    sim.set_state(torch.from_numpy(w.U0))
    sim.rk4_set_state(torch.from_numpy(w.U0))
    sim.rk4_step(4)
    sim.sync()
    e0, e1 = _events()
    e0.record()
    sim.rk4_step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    peak = float(sim.rk4_field(dp.FIELD_U).abs().max().item())
    sim.close()
    return {"workload": "2D 4096^2 + 32-cell layer (4160^2 cells), FP32, classic RK4, %d steps" % steps,
            "value": round(w.cells * steps / (ms * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "ms_per_step": round(ms / steps, 5), "finite": bool(np.isfinite(peak))}


def bench_walls(steps: int = 500):
    """The 4160^2 FP32 workload truncated by reflecting walls (Dirichlet
    ghosts) instead of the periodic wrap, autotuned launch."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    from paper_1804_01390_amd import autotune
    w = synthetic.bumps2d(n=4096, m=32, steps=steps, seed=0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32, walls=(True, True))
    sim.set_state(torch.from_numpy(w.U0))
    choice = autotune.tune(sim)
    sim.set_state(torch.from_numpy(w.U0))
    sim.step(10)
    sim.sync()
    e0, e1 = _events()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.set_timing(True)
    sim.step(50)
    roof = roofline_from_timing(sim.get_timing(), 50)
    sim.set_timing(False)
    roof["path_alg_GBps"] = round(alg_bytes_per_step(w, 4) * steps / (ms * 1e-3) / 1e9, 1)
    sim.close()
    return {"workload": "2D 4096^2 + 32-cell layer (4160^2 cells) inside reflecting walls, FP32, %d steps" % steps,
            "value": round(w.cells * steps / (ms * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "ms_per_step": round(ms / steps, 5), "roofline": roof,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": True}}


def bench_reflection(dn: str = "f64", checks=(64, 2000)):
    """The paper's claim on the 2D 4096^2 + 32 workload (its 64 bumps with
    the two cells next to each interface zeroed): the layered run in its
    tuned launch against the plain wave equation on a 6144^2 periodic grid
    with no layer (a margin of 1024 cells per side: no wave reaches its edge
    in 2000 steps), both on the GPU; max |U - U_free| over the physical
    domain, relative to the initial peak.  Before any wave can have crossed
    the 64-cell band (64 steps) the difference is rounding; after the full
    run it holds the residual the layer lets through."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    from paper_1804_01390_amd import autotune
    td = torch.float64 if dn == "f64" else torch.float32
    w = synthetic.bumps2d(n=4096, m=32, steps=max(checks), seed=0, margin=2)
    n, m, Nf = w.n[0], w.lo[0], 6144
    off = (Nf - n) // 2
    peak = float(np.max(np.abs(w.U0)))
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=td)
    sim.set_state(torch.from_numpy(w.U0))
    choice = autotune.tune(sim)
    sim.set_state(torch.from_numpy(w.U0))
    U0f = np.zeros((Nf, Nf))
    U0f[off:off + n, off:off + n] = w.U0[m:m + n, m:m + n]
    free = dp.Simulation([Nf, Nf], [0, 0], [0, 0], w.h, w.dt, [None, None], dtype=td)
    free.set_state(torch.from_numpy(U0f))
    out, done = {}, 0
    for t in checks:
        sim.step(t - done)
        free.step(t - done)
        done = t
        a = sim.U.double()[m:m + n, m:m + n]
        b = free.U.double()[off:off + n, off:off + n]
        out[str(t)] = float((a - b).abs().max().item()) / peak
    sim.close()
    free.close()
    return {"workload": "2D 4096^2 + 32-cell layer (4160^2 cells), 64 seeded bumps zero on the two cells next to "
                        "each interface, %s, tuned launch, against the plain wave equation on 6144^2 (no layer), "
                        "both on the GPU" % dn.upper(),
            "max_abs_diff_over_initial_peak": out,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": True}}


def bench_small(steps: int = 500):
    """The 128^2 + 16-cell (160^2 cells) FP64 parity workload, 500 steps: a
    step is far shorter than a kernel launch, so it measures the step loop:
    eager launches against one HIP-graph replay of the whole run."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    w = synthetic.bump2d(128, 16, steps)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    out = {"workload": "2D 128^2 + 16-cell layer (160^2 cells), FP64, %d steps" % steps}
    for mode in ("eager", "graph"):
        sim.set_state(torch.from_numpy(w.U0))
        (sim.step_graph if mode == "graph" else sim.step)(steps)    # warm (graph: capture)
        sim.set_state(torch.from_numpy(w.U0))
        sim.sync()
        e0, e1 = _events()
        e0.record()
        (sim.step_graph if mode == "graph" else sim.step)(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[mode + "_us_per_step"] = round(ms * 1e3 / steps, 3)
        out[mode + "_value"] = round(w.cells * steps / (ms * 1e-3) / 1e9, 3)
    out["unit"] = "Gcell/s"
    sim.close()
    return out


def bench_batch(steps: int, count: int):
    """``count`` independent 2D problems (sides log-uniform in [256, 1536],
    16-32-cell layers), FP32, one Gaussian each: one HIP-graph launch for the
    whole run (one kernel per step over a tile list of all problems) against
    separate runs of each problem."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    probs = synthetic.batch2d(count=count, steps=steps)
    cells = sum(w.cells for w in probs)
    from paper_1804_01390_amd import autotune
    multi = dp.MultiSimulation(probs, dtype=torch.float32)
    choice = autotune.tune_multi(multi, [w.U0 for w in probs], steps=20)
    multi.set_state([w.U0 for w in probs])
    multi.step(steps, graph=True)          # capture + instantiate + one run
    multi.sync()
    multi.set_state([w.U0 for w in probs])
    multi.sync()
    e0, e1 = _events()
    e0.record()
    multi.step(steps, graph=True)          # the cached graph: one launch
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)
    multi_tiles = multi.tiles
    multi.close()
    sims = []
    for w in probs:
        s = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
        s.set_state(torch.from_numpy(w.U0))
        sims.append(s)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for s in sims:
        s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_sep = e0.elapsed_time(e1)
    for s in sims:
        s.close()
    ab = sum(alg_bytes_per_step(w, 4) for w in probs)
    return {"workload": "%d 2D problems, sides log-uniform in [256,1536], 16-32-cell layers, FP32, "
                        "%d steps (%d cells per step)" % (count, steps, cells),
            "alg_bytes_per_step": ab,
            "graph_alg_GBps": round(ab * steps / (ms_graph * 1e-3) / 1e9, 1),
            "graph_value": round(cells * steps / (ms_graph * 1e-3) / 1e9, 3),
            "separate_value": round(cells * steps / (ms_sep * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "graph_ms": round(ms_graph, 3), "separate_ms": round(ms_sep, 3),
            "speedup": round(ms_sep / ms_graph, 3),
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "group": choice["group"],
                       "autotuned": True, "tiles": multi_tiles}}


def bench_adjoint(steps: int, shots: int):
    """2D 1024^2 + 32-cell layer, FP32 fields, smooth random c^2, ``shots``
    Ricker shots, 1024 receivers: observed traces from a second c^2, then the
    checkpointed forward and the reverse-time adjoint (FP64 gradient)."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    w = synthetic.shots2d(shots=shots, steps=steps)
    B, cells = shots, w.cells
    src = [b * cells + w.sources[b][0] for b in range(B)]
    rec = [b * cells + r for b in range(B) for r in w.receivers]

    def make(c2):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, c2=c2, dtype=torch.float32, batch=B)
        sim.set_state(torch.zeros(sim.shape, dtype=torch.float32, device="cuda"))
        sim.inject(src, torch.from_numpy(w.wavelets))
        tr = sim.record(rec, steps)
        return sim, tr

    sim, obs = make(w.c2_true)
    sim.step(steps)
    sim.sync()
    obs = obs.clone()
    sim.close()
    sim, tr = make(w.c2_model)
    from paper_1804_01390_amd import autotune
    choice = autotune.tune(sim, steps=10)      # the forward and the adjoint's recompute use it
    sim.set_state(torch.zeros(sim.shape, dtype=torch.float32, device="cuda"))
    # plain forward (no checkpoints) for reference
    sim.sync()
    e0, e1 = _events()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1)
    # the same forward in single steps (one thread per cell): the step every
    # multi-step pass is measured against
    sim.set_variant(dp.VARIANT_CELL, 4)
    sim.set_state(torch.zeros(sim.shape, dtype=torch.float32, device="cuda"))
    sim.sync()
    e0, e1 = _events()
    e0.record()
    sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1)
    sim.set_variant(choice["variant"], choice["tile_rows"])
    sim.set_state(torch.zeros(sim.shape, dtype=torch.float32, device="cuda"))
    sim.sync()
    e0, e1 = _events()
    e0.record()
    sim.forward_checkpointed(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1)
    resid = (tr - obs).contiguous()
    grad = torch.zeros(tuple(reversed(w.N)), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    gc2, gw = sim.adjoint(resid, grad_c2=grad)
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1)
    misfit = 0.5 * float((resid.double() ** 2).sum().item())
    gnorm = float(gc2.abs().max().item())
    finite = bool(torch.isfinite(gc2).all().item())
    sim.close()
    return {"workload": "2D 1024^2 + 32-cell layer (1088^2 cells) x %d shots, FP32 fields, FP64 c^2 "
                        "gradient, 1024 receivers, %d steps, sqrt(T) checkpoints" % (B, steps),
            "forward_ms": round(ms_fwd, 3), "forward_plain_ms": round(ms_plain, 3),
            "backward_ms": round(ms_bwd, 3),
            "adjoint_forward_ratio": round(ms_bwd / ms_fwd, 3),
            "forward_single_step_ms": round(ms_single, 3),
            "adjoint_single_step_ratio": round(ms_bwd / ms_single, 3),
            "forward_value": round(B * cells * steps / (ms_fwd * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "misfit": misfit, "grad_c2_max": gnorm, "grad_finite": finite,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": True}}


def bench_2d(dn: str, steps: int, warmup: int, variant: int = 0, tile_rows: int = 0):
    """The 2D 4096^2 + 32-cell workload (64 seeded Gaussians), `steps` of its
    2000 steps, tuned launch, eager or as one graph replay (the faster)."""
    import synthetic
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0)
    r = time_gpu(w, dn, steps, warmup, variant, tile_rows)
    roof = roofline_from_timing(r["kernels"], r["timed_steps"], w.name, dn)
    # the whole path: algorithmic bytes per step over the measured time per step
    # (kernels of a step may overlap on two streams, so this is not their sum)
    roof["path_alg_GBps"] = round(alg_bytes_per_step(w, 4 if dn == "f32" else 8) / (r["ms_per_step"] * 1e-3) / 1e9, 1)
    path_hbm(roof, r["kernels"], r["timed_steps"], r["ms_per_step"], w.name, dn)
    return {"dtype": dn,
            "workload": "2D 4096^2 interior + 32-cell layer per side (4160^2 cells), 64 seeded Gaussians, "
                        "%s, c=1, dt=h/2, quadratic damping ramp to 2/h; %d of the workload's 2000 steps timed "
                        "after %d warmup steps" % (dn.upper(), steps, warmup),
            "cells": w.cells, "steps": steps,
            "value": round(w.cells * steps / (r["total_ms"] * 1e-3) / 1e9, 3),
            "ms_per_step": round(r["ms_per_step"], 5), "roofline": roof, "kernels": r["kernels"],
            "finite": r["finite"], "launch": r["launch"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000,
                    help="steps timed of each single-grid workload (the 3D headline has 1000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=2)     # ~15 s of the oracle on 16 host cores
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant", type=int, default=0,
                    help="a fixed variant instead of the tuner (with --only: that record)")
    ap.add_argument("--tile-rows", type=lambda v: int(v, 0), default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the streaming bandwidth probe and exit")
    ap.add_argument("--quick", action="store_true",
                    help="only the single-grid records (skip the batched, adjoint, RK4, walls and small workloads)")
    ap.add_argument("--adjoint-steps", type=int, default=3000)
    ap.add_argument("--batch-steps", type=int, default=1500)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--only", default="",
                    help="run a single section: ricker3d, ricker3d32, bumps2d, bumps2d64, batch, adjoint, "
                         "small, rk4, walls or reflection")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the stencil would shard by slabs "
              "with halo exchange; that path is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    steps3d = min(args.steps, 1000)
    if args.only:
        fn = {"ricker3d": lambda: bench_ricker3d(steps3d, args.warmup, "f64", args.variant, args.tile_rows),
              "ricker3d32": lambda: bench_ricker3d(steps3d, args.warmup, "f32", args.variant, args.tile_rows),
              "bumps2d": lambda: bench_2d("f32", args.steps, args.warmup, args.variant, args.tile_rows),
              "bumps2d64": lambda: bench_2d("f64", args.steps, args.warmup, args.variant, args.tile_rows),
              "batch": lambda: bench_batch(args.batch_steps, args.batch_count),
              "adjoint": lambda: bench_adjoint(args.adjoint_steps, 32),
              "small": bench_small, "rk4": bench_rk4, "walls": bench_walls,
              "reflection": bench_reflection}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    import synthetic
    log("headline: 3D 560^3 FP64, %d warmup + %d steps" % (args.warmup, steps3d))
    head = bench_ricker3d(steps3d, args.warmup, "f64")
    log("  %.1f Gcell/s, %.4f ms/step; %s kernel %.4f ms/launch, %.0f GB/s algorithmic; launch %s" % (
        head["value"], head["ms_per_step"], head["roofline"]["kernel"], head["roofline"]["kernel_ms_mean"],
        head["roofline"]["achieved"], head["launch"]))
    runs = [head]
    log("3D 560^3 FP32")
    runs.append(bench_ricker3d(steps3d, args.warmup, "f32"))
    log("  %.1f Gcell/s, %.4f ms/step" % (runs[-1]["value"], runs[-1]["ms_per_step"]))
    for dn in ("f32", "f64"):
        steps2d = min(args.steps, 2000)
        log("2D 4160^2 %s: %d warmup + %d steps" % (dn, args.warmup, steps2d))
        runs.append(bench_2d(dn, steps2d, args.warmup))
        log("  %.1f Gcell/s, %.4f ms/step; launch %s" % (runs[-1]["value"], runs[-1]["ms_per_step"],
                                                        runs[-1]["launch"]))
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Gcell/s",
        "n_gpus": 1,
        "steps": steps3d,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": head["workload"], "cells": head["cells"], "steps_timed": steps3d,
                   "global_batch": 1, "parallelism": "single-gpu"},
        "roofline": head["roofline"],
        "runs": runs,
    }
    if not args.quick:
        log("small: 160^2 FP64 x 500 steps, eager vs graph")
        out["small"] = bench_small()
        log("  %s" % out["small"])
        log("batch: %d problems x %d steps" % (args.batch_count, args.batch_steps))
        out["batch"] = bench_batch(args.batch_steps, args.batch_count)
        log("  %s" % out["batch"])
        log("rk4: 4160^2 FP32")
        out["rk4"] = bench_rk4()
        log("  %s" % out["rk4"])
        log("walls: 4160^2 FP32")
        out["walls"] = bench_walls()
        log("  %s" % out["walls"])
        log("reflection: 4160^2 FP64 against 6144^2 free space")
        out["reflection"] = bench_reflection()
        log("  %s" % out["reflection"])
        log("adjoint: 32 shots x %d steps" % args.adjoint_steps)
        out["adjoint"] = bench_adjoint(args.adjoint_steps, 32)
        log("  %s" % out["adjoint"])
    if not args.no_cpu:
        log("cpu baseline: oracle, %d steps of the 3D workload" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(synthetic.ricker3d(n=512, m=24, steps=1000), args.cpu_steps)
        log("  %s" % out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
