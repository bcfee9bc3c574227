"""Throughput benchmark of the fused discrete-PML step on one MI355X.

Workload: 2D, 4096 x 4096 interior + 32-cell layer on every side (4160^2
cells), c = 1, dt = h/2, damping ramping quadratically to 2/h, initial field
a seeded sum of 64 Gaussians (widths 2-8 h) at rest.  A step is one full
pass of the method over the grid: U by leapfrog with the layer terms, and
Phi_a, Psi_a of both axes, fused in one kernel.  The default run times the
workload's 2000 steps in FP32 (the reported value) and in FP64.

Prints ONE JSON line:
  value         Gcell-updates/s (all 4160^2 cells per step, layer included)
  roofline      algorithmic bytes per step / measured kernel time vs 8 TB/s
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
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_variant(variant, tile_rows)
    sim.set_state(torch.from_numpy(w.U0))
    sim.step(warmup)
    sim.sync()
    stream = torch.cuda.current_stream()
    # whole-job throughput: exactly `steps` steps between two synchronised events
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    # per-launch duration of the step kernel: one event pair per step
    # (a step of this workload is exactly one kernel launch)
    k = min(steps, 200)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    evs[0].record(stream)
    for i in range(k):
        sim.step(1)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(k)]
    ok = bool(np.isfinite(sim.U.float().abs().max().item()))
    sim.close()
    return {"total_ms": total_ms, "ms_per_step": total_ms / steps,
            "kernel_ms_mean": float(np.mean(per)), "kernel_ms_median": float(np.median(per)),
            "finite": ok}


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


def traffic_from_profile(workload: str, dtype_name: str):
    """HBM bytes per launch measured by rocprofv3 counters, if a summary for
    this kernel source is committed under profiles/."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, dtype_name))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time a plain 1 GiB device copy and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the stencil would shard by slabs "
              "with halo exchange; that path is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import synthetic
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0)
    runs = []
    for dn in args.dtypes.split(","):
        log("timing %s %s: %d warmup + %d steps" % (w.name, dn, args.warmup, args.steps))
        r = time_gpu(w, dn, args.steps, args.warmup, args.variant, args.tile_rows)
        esize = 4 if dn == "f32" else 8
        ab = alg_bytes_per_step(w, esize)
        achieved = ab / (r["kernel_ms_mean"] * 1e-3) / 1e9
        traffic = traffic_from_profile(w.name, dn)
        runs.append({
            "dtype": dn,
            "value": round(w.cells * args.steps / (r["total_ms"] * 1e-3) / 1e9, 3),
            "ms_per_step": round(r["ms_per_step"], 5),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": traffic,
                         "alg_bytes_per_launch": ab,
                         "kernel_ms_mean": round(r["kernel_ms_mean"], 5),
                         "kernel_ms_median": round(r["kernel_ms_median"], 5)},
            "finite": r["finite"],
        })
        log("  %s: %.1f Gcell/s, %.4f ms/step, kernel %.4f ms, %.0f GB/s" % (
            dn, runs[-1]["value"], r["ms_per_step"], r["kernel_ms_mean"], achieved))
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
    if not args.no_cpu:
        log("cpu baseline: oracle, %d steps" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
