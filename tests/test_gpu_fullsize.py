"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (autotuned variant).  Where the oracle cannot run the whole
workload it checks sampled outputs one step at a time from the GPU's own
state, or a property that holds at any size."""
import math
import time

import numpy as np
import pytest

import oracle
import synthetic
from helpers import compare_states, gpu_state, rel_err

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


def _log(msg):
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


def _bench_sim(w, dtype):
    from paper_1804_01390_amd import autotune
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_state(torch.from_numpy(w.U0))
    choice = autotune.tune(sim)
    _log("launch variant=%d tile_rows=%d" % (choice["variant"], choice["tile_rows"]))
    sim.set_state(torch.from_numpy(w.U0))
    return sim


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_bumps2d_full_size_short_run_and_last_step(dtype):
    """4160^2 cells: 20 steps against the full-grid oracle; then the GPU runs
    on to step 2000 and its last step is checked against one oracle step
    taken from the GPU's own state at step 1999."""
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0)
    _log("bumps2d 4160^2 %s" % dtype)
    sim = _bench_sim(w, dtype)
    sim.step(20)
    gs = gpu_state(sim)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    ref, _ = oracle.run(g, oracle.start(g, w.U0), 20)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    errs = compare_states(gs, ref, w.n, w.lo, w.hi)
    _log("20 steps: %s" % {k: "%.2e" % v for k, v in errs.items()})
    assert max(errs.values()) <= tol
    sim.step(1999 - 20)
    s1999 = gpu_state(sim)
    sim.step(1)
    s2000 = gpu_state(sim)
    one = oracle.step(g, s1999)
    errs = compare_states(s2000, one, w.n, w.lo, w.hi)
    # one step from a state stored in dtype: rounding of one step only
    _log("last step: %s" % {k: "%.2e" % v for k, v in errs.items()})
    assert max(errs.values()) <= (1e-14 if dtype == torch.float64 else 1e-6)
    sim.close()


def test_bumps2d_full_size_fp64_full_run_bit_identical():
    """The whole 2000-step FP64 run of the 4160^2 workload equals the oracle's
    (h = 1 and dt = 1/2 are powers of two and both sides evaluate the scheme
    in the same operation order)."""
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0)
    sim = _bench_sim(w, torch.float64)
    sim.step(2000)
    gs = gpu_state(sim)
    sim.close()
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    s = oracle.start(g, w.U0)
    for k in range(10):
        s, _ = oracle.run(g, s, 200)
        _log("oracle %d / 2000" % s.n)
    errs = compare_states(gs, s, w.n, w.lo, w.hi)
    _log("2000 steps: %s; bit-identical U: %s" % ({k: "%.2e" % v for k, v in errs.items()},
                                                  bool(np.array_equal(gs.U, s.U))))
    assert max(errs.values()) <= 1e-12


def _sub_box(state, g, w, start, size):
    """Oracle one-step of a periodic sub-box (gathered with wrapped indices);
    valid on the box's interior (one cell in from its faces)."""
    nd = len(start)
    idx = [(np.arange(size[a]) + start[a]) % w.N[a] for a in range(nd)]
    ix = np.ix_(*reversed(idx))                         # numpy axes are z, y, x

    def cut(a):
        return np.ascontiguousarray(a[ix])

    sig = [np.ascontiguousarray(w.sigma[a][idx[a]]) for a in range(nd)]
    sub = oracle.State(cut(state.U), cut(state.Uprev), [cut(p) for p in state.Phi], [cut(p) for p in state.Psi])
    gg = oracle.Grid(list(size), g.h, g.dt, sig)
    return oracle.step(gg, sub), cut


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_ricker3d_full_size_sampled_steps(dtype):
    """560^3 cells, Ricker source and plane recorder, autotuned launch: after
    700 steps (the wave, 0.4 cells per step, has crossed the 256 cells to the
    layer and is inside it), one GPU step is checked on sampled sub-boxes
    (interior, the six layer faces, an edge, a corner and the box around the
    source) against oracle steps taken from the GPU's own state."""
    from paper_1804_01390_amd import autotune
    steps = 700
    w = synthetic.ricker3d(n=512, m=24, steps=1000)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=dtype, device="cuda"))
    sim.inject(w.sources, torch.from_numpy(w.wavelets))
    axis, index = w.plane
    planes = sim.record_plane(axis, index, w.steps)
    choice = autotune.tune(sim, steps=10)
    _log("launch variant=%d tile_rows=%d" % (choice["variant"], choice["tile_rows"]))
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=dtype, device="cuda"))
    sim.step(steps)
    before = gpu_state(sim)
    sim.step(1)
    after = gpu_state(sim)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    m, n = 24, 512
    size = [20, 20, 20]
    c = m + n // 2
    starts = [[c - 10, c - 10, c - 10],            # source
              [300, 200, 100],                     # interior
              [n + m - 6, 200, 300], [m - 14, 250, 260],        # x layer, both sides
              [250, n + m - 6, 250], [260, m - 14, 240],        # y layer
              [250, 260, n + m - 6], [240, 250, m - 14],        # z layer
              [n + m + 10, n + m + 10, 250],       # an edge of the layer
              [550, 550, 550]]                     # the corner across the periodic wrap
    worst = 0.0
    peak = float(np.max(np.abs(after.U)))
    for st in starts:
        one, cut = _sub_box(before, g, w, st, size)
        inner = (slice(1, -1),) * 3
        got = cut(after.U)
        worst = max(worst, float(np.max(np.abs(got[inner] - one.U[inner]))) / peak)
        for a in range(3):
            M = w.lo[a] + w.hi[a]
            jj = (((np.arange(size[a]) + st[a]) % w.N[a]) - (w.lo[a] + w.n[a])) % w.N[a]   # band slot
            for kind, arr, ref in (("phi", after.Phi[a], one.Phi[a]), ("psi", after.Psi[a], one.Psi[a])):
                on = (jj <= M - 1) if kind == "phi" else ((jj >= 1) & (jj <= M))
                shape = [1, 1, 1]
                shape[2 - a] = size[a]
                mm = np.broadcast_to(on.reshape(shape), tuple(reversed(size)))[inner]
                sub = cut(arr)
                if mm.any():
                    worst = max(worst, float(np.max(np.abs(sub[inner][mm] - ref[inner][mm]))) / max(peak, 1e-30))
    # the recorded plane of the last step equals the field on that plane
    pl = planes[steps].double().cpu().numpy()
    assert np.array_equal(pl, after.U[index].astype(np.float64))
    _log("sampled one-step error / peak: %.2e" % worst)
    assert worst <= (1e-6 if dtype == torch.float32 else 1e-12)
    lay = max(float(np.max(np.abs(p))) for p in after.Phi + after.Psi)
    _log("largest layer field / peak: %.2e" % (lay / peak))
    assert lay > 1e-6 * peak                                 # the layer is active
    sim.close()


def test_ricker3d_full_size_fp64_headline_launch():
    """The benchmark's headline workload as the benchmark runs it: 560^3
    cells, FP64, the Ricker source at the centre, the z plane through it
    recorded, the tuned launch (two-step passes with the source added inside
    the core).  After 25 steps from rest (twelve passes and one single step)
    every cell of U, U^{n-1}, Phi and Psi is compared with the oracle's run of
    the same 25 steps, and the recorded plane after steps 8, 16 and 24 with
    the oracle's field on that plane."""
    from paper_1804_01390_amd import autotune
    w = synthetic.ricker3d(n=512, m=24, steps=1000)
    zeros = lambda: torch.zeros(tuple(reversed(w.N)), dtype=torch.float64, device="cuda")
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    sim.set_state(zeros())
    sim.inject(w.sources, torch.from_numpy(w.wavelets))
    axis, index = w.plane
    planes = sim.record_plane(axis, index, w.steps)
    choice = autotune.tune(sim, steps=10)
    _log("launch variant=%d tile_rows=0x%x" % (choice["variant"], choice["tile_rows"]))
    sim.set_state(zeros())
    sim.step(25)
    gs = gpu_state(sim)
    pl = sim._keep["planes"].cpu().numpy()
    sim.close()
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    s = oracle.start(g, np.zeros(tuple(reversed(w.N))))
    nt = w.wavelets.shape[1]
    done = 0
    for t in (8, 16, 24, 25):
        s, _ = oracle.run(g, s, t - done, sources=w.sources, wavelets=w.wavelets, nt=nt)
        done = t
        _log("oracle at step %d" % t)
        if t < 25:
            err = rel_err(pl[t - 1], s.U[index])
            _log("plane after step %d: error / peak %.2e" % (t, err))
            assert err <= 1e-12
    errs = compare_states(gs, s, w.n, w.lo, w.hi)
    _log("errors: %s" % {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= 1e-12, (k, v)


def test_batch_full_size_sampled_problems():
    """The 256-problem batch in the benchmark's launch (tuned scheme and shape,
    graph launch): the three smallest problems run all 1500 steps against the
    oracle; three others are checked one step from the GPU state after 1500
    steps."""
    from paper_1804_01390_amd import autotune
    probs = synthetic.batch2d(count=256, steps=1500)
    sim = dp.MultiSimulation(probs, dtype=torch.float32)
    choice = autotune.tune_multi(sim, [w.U0 for w in probs], steps=20)
    _log("launch variant=%d tile_rows=%d group=%d" % (choice["variant"], choice["tile_rows"], choice["group"]))
    sim.set_state([w.U0 for w in probs])
    sim.step(1499, graph=True)
    sim.sync()
    order = np.argsort([w.cells for w in probs])
    small, other = list(order[:3]), [int(order[128]), int(order[200]), int(order[-1])]
    before = {}
    for i in other:
        st = oracle.State(sim.field(i, dp.FIELD_U).double().cpu().numpy(),
                          sim.field(i, dp.FIELD_UPREV).double().cpu().numpy(), [], [])
        from helpers import expand_aux
        w = probs[i]
        st.Phi = [expand_aux(sim.field(i, dp.FIELD_PHI(a)).double().cpu().numpy(), a, w.n, w.lo, w.hi, "phi")
                  for a in range(2)]
        st.Psi = [expand_aux(sim.field(i, dp.FIELD_PSI(a)).double().cpu().numpy(), a, w.n, w.lo, w.hi, "psi")
                  for a in range(2)]
        before[i] = st
    sim.step(1, graph=False)
    sim.sync()
    from helpers import compare_states, multi_state, run_with_peaks
    for i in small:
        w = probs[i]
        g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
        ref, _, peaks = run_with_peaks(g, oracle.start(g, w.U0), 1500, w.n, w.lo, w.hi)
        errs = compare_states(multi_state(sim, i, w), ref, w.n, w.lo, w.hi, peaks)
        _log("problem %d (%dx%d) full run err / run peak %s" % (i, w.N[0], w.N[1],
                                                              {k: "%.2e" % v for k, v in errs.items()}))
        for k, v in errs.items():
            assert v <= 2e-5, (i, k, v)
    for i in other:
        w = probs[i]
        g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
        one = oracle.step(g, before[i])
        got = multi_state(sim, i, w)
        # one FP32 step from the GPU's own state: errors relative to each field's peak
        errs = compare_states(got, one, w.n, w.lo, w.hi)
        _log("problem %d (%dx%d) last step err %s" % (i, w.N[0], w.N[1], {k: "%.2e" % v for k, v in errs.items()}))
        for k, v in errs.items():
            if k != "Uprev":
                assert v <= 1e-6, (i, k, v)
    sim.close()


def test_adjoint_full_size_dot_product_and_direction():
    """1088^2 cells x 32 shots, 3000 steps (the adjoint workload), FP64:
    the wavelet gradient satisfies the dot-product identity of the linear
    wavelet-to-trace map, and the c^2 gradient matches a central difference
    along a smooth direction."""
    w = synthetic.shots2d(shots=32, steps=3000)
    B, cells, nt = 32, w.cells, w.steps
    src = [b * cells + w.sources[b][0] for b in range(B)]
    rec = [b * cells + r for b in range(B) for r in w.receivers]

    def forward(c2, wav, keep=False):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, c2=c2, dtype=torch.float64, batch=B)
        sim.set_state(torch.zeros(sim.shape, dtype=torch.float64, device="cuda"))
        sim.inject(src, torch.as_tensor(wav))
        tr = sim.record(rec, nt)
        if keep:
            sim.forward_checkpointed(nt)
        else:
            sim.step(nt)
        sim.sync()
        return sim, tr.clone()

    rng = np.random.default_rng(3)
    y = rng.normal(size=(B * len(w.receivers), nt))
    sim, tr = forward(w.c2_model, w.wavelets, keep=True)
    _, gw = sim.adjoint(torch.from_numpy(y))
    sim.sync()
    lhs = float((tr.cpu().numpy() * y).sum())           # <F w, y>, F linear in w
    rhs = float((w.wavelets * gw.cpu().numpy()).sum())  # <w, F^T y>
    _log("dot product: %.15e vs %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    sim.close()
    # c^2 gradient along a smooth direction held at 0 near the layer
    obs = forward(w.c2_true, w.wavelets)[1].cpu().numpy()
    sim, tr = forward(w.c2_model, w.wavelets, keep=True)
    resid = tr.cpu().numpy() - obs
    g, _ = sim.adjoint(torch.from_numpy(resid))
    sim.sync()
    d = synthetic.smooth_c2(w.n, w.lo, w.hi, 4, 60.0, 120.0, 1.0, 12, np.random.default_rng(9)) - 1.0
    ad = float((g.cpu().numpy() * d).sum())
    sim.close()
    eps = 1e-4

    def J(c2):
        s, t = forward(c2, w.wavelets)
        s.close()
        return 0.5 * float(((t.cpu().numpy() - obs) ** 2).sum())

    fd = (J(w.c2_model + eps * d) - J(w.c2_model - eps * d)) / (2 * eps)
    _log("directional derivative: adjoint %.10e, central difference %.10e" % (ad, fd))
    assert abs(ad - fd) <= 1e-5 * abs(fd)
