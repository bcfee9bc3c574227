"""Throughput benchmark of the fused discrete-PML step on one MI355X.

Workload: 2D, 4096 x 4096 interior + 32-cell layer on every side (4160^2
cells), c = 1, dt = h/2, damping ramping quadratically to 2/h, initial field
a seeded sum of 64 Gaussians (widths 2-8 h) at rest.  A step is one full
pass of the method over the grid: U by leapfrog with the layer terms, and
Phi_a, Psi_a of both axes, fused in one kernel.  The default run times the
workload's 2000 steps in FP32 (the reported value) and in FP64.

Prints ONE JSON line:
  value         Gcell-updates/s (all 4160^2 cells per step, layer included)
  roofline      the dominant step kernel: algorithmic bytes per launch over its
                mean launch duration (HIP events around each launch, on the
                library's stream) vs 8 TB/s
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload

    python bench.py [--gpus 1] [--steps 2000] [--warmup 50]
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


def roofline_from_timing(kernels, timed_steps):
    """Roofline of the dominant step kernel from the library's per-launch
    timing: its algorithmic bytes per launch over its mean launch duration.
    The dominant kernel is the class that moves the most algorithmic bytes:
    frame launches run on a second stream beside the core, so their event
    durations include time spent sharing the GPU and are no measure of which
    kernel carries the step."""
    name, k = max(((n, v) for n, v in kernels.items() if v["launches"]), key=lambda kv: kv[1]["bytes"])
    ms = k["ms"] / k["launches"]
    bpl = k["bytes"] / k["launches"]
    achieved = bpl / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": name,
            "alg_bytes_per_launch": int(round(bpl)), "kernel_ms_mean": round(ms, 5),
            "launches": k["launches"], "timed_steps": timed_steps}


def cpu_baseline(w, sample_steps: int):
    """The FP64 oracle on the same workload for `sample_steps` steps."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    s = oracle.start(g, w.U0)
    oracle.run(g, s, 1)            # page in, spin up threads
    t = time.perf_counter()
    oracle.run(g, s, sample_steps)
    dt = time.perf_counter() - t
    return {"value": round(sample_steps * w.cells / dt / 1e9, 5), "unit": "Gcell/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d steps of the same %dx%d-cell workload, FP64, OpenMP over cells"
                      % (sample_steps, w.N[0], w.N[1]),
            "seconds": round(dt, 3)}


def traffic_from_profile(workload: str, dtype_name: str, kernel: str):
    """HBM bytes per launch of a step-kernel class measured by rocprofv3
    counters, if a summary for this kernel source is committed under profiles/."""
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
    return rec.get("bytes_per_launch")


def copy_probe(mib: int = 1024, reps: int = 20):
    """A plain device copy of known size (torch's copy kernel): the achievable
    read+write bandwidth on this GPU and the reference for scaling the HBM
    counters of rocprofv3 (FETCH_SIZE / WRITE_SIZE) to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "ms": round(ms, 4), "GB_per_s": round(gbs, 1)}), flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_ricker3d(steps: int):
    """3D, 512^3 interior + 24-cell layer on all faces (560^3 cells), FP32,
    dt = 0.4 h, Ricker point source at the centre, the z plane through it
    recorded every step."""
    import torch
    import paper_1804_01390_amd as dp
    import synthetic
    from paper_1804_01390_amd import autotune
    w = synthetic.ricker3d(n=512, m=24, steps=steps)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=torch.float32, device="cuda"))
    sim.inject(w.sources, torch.from_numpy(w.wavelets))
    axis, index = w.plane
    sim.record_plane(axis, index, w.steps)
    choice = autotune.tune(sim, steps=10)
    sim.step(5)
    sim.sync()
    e0, e1 = _events()
    # restart from rest so the timed run is the workload's steps 0..steps-1
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=torch.float32, device="cuda"))
    sim.sync()
    e0.record()
    sim.step(w.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    plane_cells = w.N[0] * w.N[1]
    ab = alg_bytes_per_step(w, 4) + plane_cells * 4
    peak = float(sim._keep["planes"][-1].abs().max().item())
    # the step kernel alone (library launch timing), on a restarted run
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=torch.float32, device="cuda"))
    sim.set_timing(True)
    sim.step(50)
    roof = roofline_from_timing(sim.get_timing(), 50)
    sim.set_timing(False)
    roof["traffic"] = traffic_from_profile("ricker3d_512_m24", "f32", roof["kernel"])
    roof["path_alg_GBps"] = round(ab * w.steps / (ms * 1e-3) / 1e9, 1)
    sim.close()
    return {"workload": "3D 512^3 interior + 24-cell layer (560^3 cells), FP32, Ricker source, "
                        "plane recorded every step, %d steps" % w.steps,
            "value": round(w.cells * w.steps / (ms * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "ms_per_step": round(ms / w.steps, 5),
            "alg_GBps": round(ab * w.steps / (ms * 1e-3) / 1e9, 1),
            "frac_of_8TBps": round(ab * w.steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "last_plane_peak": peak, "roofline": roof,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": True}}


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
            "forward_value": round(B * cells * steps / (ms_fwd * 1e-3) / 1e9, 3), "unit": "Gcell/s",
            "misfit": misfit, "grad_c2_max": gnorm, "grad_finite": finite,
            "launch": {"variant": choice["variant"], "tile_rows": choice["tile_rows"], "autotuned": True}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=160)   # ~10 s of the oracle on 16 host cores
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 1 GiB device copy and exit")
    ap.add_argument("--quick", action="store_true",
                    help="only the 4160^2 workload (skip the 3D, batched and adjoint workloads)")
    ap.add_argument("--adjoint-steps", type=int, default=3000)
    ap.add_argument("--batch-steps", type=int, default=1500)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--steps-3d", type=int, default=1000)
    ap.add_argument("--only", default="",
                    help="run a single section: ricker3d, batch, adjoint, small, rk4 or walls")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the stencil would shard by slabs "
              "with halo exchange; that path is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.only:
        fn = {"ricker3d": lambda: bench_ricker3d(args.steps_3d),
              "batch": lambda: bench_batch(args.batch_steps, args.batch_count),
              "adjoint": lambda: bench_adjoint(args.adjoint_steps, 32),
              "small": bench_small, "rk4": bench_rk4, "walls": bench_walls}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    import synthetic
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0)
    runs = []
    for dn in args.dtypes.split(","):
        log("timing %s %s: %d warmup + %d steps" % (w.name, dn, args.warmup, args.steps))
        r = time_gpu(w, dn, args.steps, args.warmup, args.variant, args.tile_rows)
        roof = roofline_from_timing(r["kernels"], r["timed_steps"])
        roof["traffic"] = traffic_from_profile(w.name, dn, roof["kernel"])
        # the whole path: algorithmic bytes per step over the measured time per step
        # (kernels of a step may overlap on two streams, so this is not their sum)
        roof["path_alg_GBps"] = round(alg_bytes_per_step(w, 4 if dn == "f32" else 8) / (r["ms_per_step"] * 1e-3) / 1e9, 1)
        runs.append({
            "dtype": dn,
            "value": round(w.cells * args.steps / (r["total_ms"] * 1e-3) / 1e9, 3),
            "ms_per_step": round(r["ms_per_step"], 5),
            "roofline": roof,
            "kernels": r["kernels"],
            "finite": r["finite"],
            "launch": r["launch"],
        })
        log("  %s: %.1f Gcell/s, %.4f ms/step; %s kernel %.4f ms/launch, %.0f GB/s algorithmic (path %.0f GB/s)" % (
            dn, runs[-1]["value"], r["ms_per_step"], roof["kernel"], roof["kernel_ms_mean"], roof["achieved"],
            roof["path_alg_GBps"]))
        log("  launch %s" % r["launch"])
    main_run = runs[0]
    out = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "Gcell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_run["dtype"],
        "data": "synthetic",
        "config": {"workload": "2D 4096^2 interior + 32-cell layer per side (4160^2 cells), "
                               "64 seeded Gaussians, c=1, dt=h/2, quadratic damping ramp to 2/h, "
                               "2000 steps",
                   "cells": w.cells, "global_batch": 1, "parallelism": "single-gpu"},
        "roofline": main_run["roofline"],
        "runs": runs,
    }
    if not args.quick:
        log("small: 160^2 FP64 x 500 steps, eager vs graph")
        out["small"] = bench_small()
        log("  %s" % out["small"])
        log("ricker3d: %d steps" % args.steps_3d)
        out["ricker3d"] = bench_ricker3d(args.steps_3d)
        log("  %s" % out["ricker3d"])
        log("batch: %d problems x %d steps" % (args.batch_count, args.batch_steps))
        out["batch"] = bench_batch(args.batch_steps, args.batch_count)
        log("  %s" % out["batch"])
        log("rk4: 4160^2 FP32")
        out["rk4"] = bench_rk4()
        log("  %s" % out["rk4"])
        log("walls: 4160^2 FP32")
        out["walls"] = bench_walls()
        log("  %s" % out["walls"])
        log("adjoint: 32 shots x %d steps" % args.adjoint_steps)
        out["adjoint"] = bench_adjoint(args.adjoint_steps, 32)
        log("  %s" % out["adjoint"])
    if not args.no_cpu:
        log("cpu baseline: oracle, %d steps" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
