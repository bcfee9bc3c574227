"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  Tolerances (peak-normalised max error per field):
1e-12 in FP64, 2e-5 in FP32.  Auxiliaries are compared on their supports."""
import math

import numpy as np
import pytest

import oracle
import synthetic
from helpers import compare_states, gpu_state, rel_err, run_with_peaks

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


def _dtype(name):
    return torch.float64 if name == "f64" else torch.float32


def _run_both(n, lo, hi, sigma, U0, steps, dtype, variant=dp.VARIANT_AUTO, c2=None, dt=0.5, h=1.0,
              V0=None, tile_rows=0):
    print("case n=%s lo=%s hi=%s steps=%d %s variant=%d" % (n, lo, hi, steps, dtype, variant), flush=True)
    N = [lo[a] + n[a] + hi[a] for a in range(len(n))]
    sim = dp.Simulation(n, lo, hi, h, dt, sigma, c2=1.0 if c2 is None else c2, dtype=_dtype(dtype))
    sim.set_variant(variant, tile_rows)
    sim.set_state(torch.from_numpy(U0), None if V0 is None else torch.from_numpy(V0))
    sim.step(steps)
    gs = gpu_state(sim)
    g = oracle.Grid(N, h, dt, sigma, c2=c2)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0, V0), steps, n, lo, hi)
    sim.close()
    return compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None)


def _assert_errs(errs, dtype):
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= TOL[dtype], (k, v)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant", [dp.VARIANT_CELL, dp.VARIANT_MARCH])
def test_bump2d_parity(dtype, variant):
    """128^2 interior + 16-cell layer, quadratic ramp to 2, Gaussian width 4,
    dt = 0.5, 500 steps (the small FP64 parity workload)."""
    w = synthetic.bump2d(128, 16, 500)
    errs = _run_both(w.n, w.lo, w.hi, w.sigma, w.U0, w.steps, dtype, variant)
    _assert_errs(errs, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant,tile_rows", [(dp.VARIANT_CELL, 0), (dp.VARIANT_CELL, 1), (dp.VARIANT_CELL, 8),
                                               (dp.VARIANT_MARCH, 0), (dp.VARIANT_MARCH, 7),
                                               (dp.VARIANT_MARCH1, 5)])
def test_ragged_2d_random_damping(dtype, variant, tile_rows):
    """Odd extents (several tiles plus ragged tails), unequal sides, one side
    without a layer, random damping (Fig. 3 profile), white-noise data."""
    rng = np.random.default_rng(21)
    n, lo, hi = [611, 203], [5, 9], [13, 0]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(2)]
    U0 = synthetic.white_noise_disk(n, lo, hi, 60.0, 0.25, rng)
    errs = _run_both(n, lo, hi, sig, U0, 150, dtype, variant, tile_rows=tile_rows)
    _assert_errs(errs, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_axis_without_layer_and_odd_width(dtype):
    """x has no layer at all (plain periodic), y has a one-sided layer; odd row
    length (vector width falls back to 1)."""
    rng = np.random.default_rng(3)
    n, lo, hi = [257, 100], [0, 0], [0, 12]
    sig = [None, synthetic.sigma_ramp(n[1], 0, 12, 2.0)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 8, 2.0, 6.0, rng)
    errs = _run_both(n, lo, hi, sig, U0, 120, dtype, dp.VARIANT_MARCH)
    _assert_errs(errs, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant,tile_rows", [(dp.VARIANT_CELL, 4), (dp.VARIANT_CELL, 2),
                                               (dp.VARIANT_MARCH, 0), (dp.VARIANT_MARCH, 9),
                                               (dp.VARIANT_MARCH1, 7)])
def test_3d_parity(dtype, variant, tile_rows):
    rng = np.random.default_rng(8)
    n, lo, hi = [45, 38, 33], [6, 3, 7], [4, 8, 5]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(3)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 6, 2.0, 5.0, rng)
    errs = _run_both(n, lo, hi, sig, U0, 80, dtype, variant, dt=0.4, tile_rows=tile_rows)
    _assert_errs(errs, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant,tile_rows", [(dp.VARIANT_MARCH, 5), (dp.VARIANT_MARCH1, 0)])
@pytest.mark.parametrize("shape,walls", [("wide", (False, False, False)), ("wide", (True, True, True)),
                                         ("x128", (False, False, False)), ("x128", (True, False, True))])
def test_3d_march_strips_and_edges(dtype, variant, tile_rows, shape, walls):
    """3D marching waves across several 64-column strips (lanes 0 and 63 read
    the columns beyond their strip), an x extent that is a multiple of 64 (the
    last strip ends on the grid's edge), ragged row groups, with and without
    reflecting walls."""
    rng = np.random.default_rng(81)
    if shape == "wide":
        n, lo, hi = [150, 23, 14], [7, 4, 3], [6, 5, 4]
    else:
        n, lo, hi = [118, 13, 12], [4, 3, 5], [6, 2, 3]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(3)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 5, 2.0, 5.0, rng)
    N = [lo[a] + n[a] + hi[a] for a in range(3)]
    steps, dt = 50, 0.4
    print("case 3d strips %s walls=%s %s variant=%d rows=%d" % (shape, walls, dtype, variant, tile_rows), flush=True)
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, dtype=_dtype(dtype), walls=walls)
    sim.set_variant(variant, tile_rows)
    sim.set_state(torch.from_numpy(U0))
    sim.step(steps)
    gs = gpu_state(sim)
    g = oracle.Grid(N, 1.0, dt, sig, walls=walls)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
    sim.close()
    _assert_errs(compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_field_and_initial_velocity(dtype):
    rng = np.random.default_rng(5)
    n, lo, hi = [200, 150], [10, 10], [10, 10]
    sig = [synthetic.sigma_ramp(n[a], 10, 10, 2.0) for a in range(2)]
    c2 = synthetic.smooth_c2(n, lo, hi, 6, 10.0, 30.0, 0.5, 8, rng)
    U0 = synthetic.gaussian_sum(n, lo, hi, 10, 2.0, 6.0, rng)
    V0 = synthetic.gaussian_sum(n, lo, hi, 10, 2.0, 6.0, rng)
    dt = 0.5 / math.sqrt(float(np.max(c2)))
    errs = _run_both(n, lo, hi, sig, U0, 200, dtype, dp.VARIANT_MARCH, c2=c2, dt=dt, V0=V0)
    _assert_errs(errs, dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sources_receivers_plane_3d(dtype):
    """Ricker point source at the centre, point receivers and a recorded
    plane through the source."""
    w = synthetic.ricker3d(n=40, m=6, steps=90, ppw=8.0)
    w.sources.append(synthetic.flat_index(w.N, [10, 12, 30]))
    wav = np.vstack([w.wavelets, 0.5 * np.roll(w.wavelets[0], 7)[None, :]])
    rec = [w.sources[0], synthetic.flat_index(w.N, [3, 3, 3]), synthetic.flat_index(w.N, [30, 25, 20]),
           w.sources[1]]
    print("case ricker3d n=40 m=6 steps=90 %s" % dtype, flush=True)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=_dtype(dtype))
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=torch.float64))
    sim.inject(w.sources, torch.from_numpy(wav))
    tr = sim.record(rec, w.steps)
    axis, index = w.plane
    pl = sim.record_plane(axis, index, w.steps)
    sim.step(w.steps)
    gs = gpu_state(sim)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    ref, rtr = oracle.run(g, oracle.start(g, np.zeros(tuple(reversed(w.N)))), w.steps,
                          sources=w.sources, wavelets=wav, receivers=rec, nt=w.steps)
    errs = compare_states(gs, ref, w.n, w.lo, w.hi)
    errs["traces"] = rel_err(tr.double().cpu().numpy(), rtr)
    # plane at the final step must equal the final field on that plane
    errs["plane_final"] = rel_err(pl[-1].double().cpu().numpy(), ref.U[index])
    sim.close()
    _assert_errs(errs, dtype)


def test_plane_recorder_matches_oracle_every_step():
    w = synthetic.ricker3d(n=24, m=4, steps=30, ppw=6.0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    sim.set_state(torch.zeros(tuple(reversed(w.N)), dtype=torch.float64))
    sim.inject(w.sources, torch.from_numpy(w.wavelets))
    axis, index = w.plane
    pl = sim.record_plane(axis, index, w.steps).cpu()
    sim.step(w.steps)
    sim.sync()
    pl = sim._keep["planes"].double().cpu().numpy()
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    s = oracle.start(g, np.zeros(tuple(reversed(w.N))))
    for k in range(w.steps):
        s, _ = oracle.run(g, s, 1, sources=w.sources, wavelets=w.wavelets, nt=w.steps)
        assert rel_err(pl[k], s.U[index]) <= 1e-12, k
    sim.close()


def test_checkpoint_resume_is_bit_identical():
    w = synthetic.bump2d(96, 12, 0)
    runs = []
    for resume in (False, True):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
        sim.set_state(torch.from_numpy(w.U0))
        sim.step(77)
        if resume:
            blob, n = sim.get_state()
            blob = blob.clone()
            sim.close()
            sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
            sim.put_state(blob, n)
        sim.step(123)
        sim.sync()
        runs.append(gpu_state(sim))
        assert sim.time_index == 200
        sim.close()
    a, b = runs
    assert np.array_equal(a.U, b.U) and np.array_equal(a.Uprev, b.Uprev)
    for k in range(2):
        assert np.array_equal(a.Phi[k], b.Phi[k]) and np.array_equal(a.Psi[k], b.Psi[k])


def test_runs_are_deterministic():
    w = synthetic.bumps2d(n=700, m=20, steps=60, seed=4)
    out = []
    for _ in range(2):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
        sim.set_state(torch.from_numpy(w.U0))
        sim.step(w.steps)
        sim.sync()
        out.append(sim.U.cpu().numpy().copy())
        sim.close()
    assert np.array_equal(out[0], out[1])


def test_step_checked_reports_nonfinite():
    w = synthetic.bump2d(64, 8, 0)
    U0 = w.U0.copy()
    U0[40, 40] = np.nan
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    sim.set_state(torch.from_numpy(U0))
    with pytest.raises(dp.DpmlError) as ei:
        sim.step_checked(20, 5)
    assert ei.value.code == dp.DPML_ENONFINITE
    sim.close()
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    sim.set_state(torch.from_numpy(w.U0))
    sim.step_checked(20, 5)
    assert sim.time_index == 20
    sim.close()


def test_set_variant_rejects_bad_shapes():
    w = synthetic.bump2d(32, 4, 0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    for variant, tile_rows in [(8, 0), (-1, 0), (dp.VARIANT_TWOSTEP, 1 << 20), (dp.VARIANT_DEEP, 1 << 20),
                               (dp.VARIANT_DEEP, 9 << 20), (dp.VARIANT_DEEP, 1 << 25), (dp.VARIANT_CELL, -1)]:
        with pytest.raises(dp.DpmlError) as ei:
            sim.set_variant(variant, tile_rows)
        assert ei.value.code == dp.DPML_EINVAL
    sim.set_variant(dp.VARIANT_DEEP, (8 << 20) | (4 << 12) | 16)
    sim.close()


def test_step_before_state_is_an_error():
    w = synthetic.bump2d(32, 4, 0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    with pytest.raises(dp.DpmlError) as ei:
        sim.step(1)
    assert ei.value.code == dp.DPML_ESTATE
    sim.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim,variant,walls", [
    (2, dp.VARIANT_CELL, (True, True)), (2, dp.VARIANT_MARCH, (True, True)),
    (2, dp.VARIANT_MARCH, (True, False)), (2, dp.VARIANT_MARCH, (False, True)),
    (3, dp.VARIANT_CELL, (True, True, True)), (3, dp.VARIANT_MARCH, (True, False, True)),
])
def test_reflecting_walls_match_oracle(dtype, ndim, variant, walls):
    """Layers truncated by reflecting walls (ghost cells hold 0) instead of the
    periodic wrap; long enough for the wall echo to return."""
    rng = np.random.default_rng(44)
    if ndim == 2:
        n, lo, hi, steps, dt = [170, 121], [7, 12], [10, 5], 160, 0.5
    else:
        n, lo, hi, steps, dt = [34, 27, 23], [5, 3, 6], [4, 7, 5], 60, 0.4
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(ndim)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 6, 2.0, 6.0, rng)
    N = [lo[a] + n[a] + hi[a] for a in range(ndim)]
    print("case walls=%s %dD %s variant=%d" % (walls, ndim, dtype, variant), flush=True)
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, dtype=_dtype(dtype), walls=walls)
    sim.set_variant(variant, 0)
    sim.set_state(torch.from_numpy(U0))
    sim.step(steps)
    gs = gpu_state(sim)
    g = oracle.Grid(N, 1.0, dt, sig, walls=walls)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
    sim.close()
    _assert_errs(compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_graph_replay_matches_eager(dtype):
    """Steps replayed from a captured HIP graph: every replay (with eager work
    and synchronisations between replays) equals eager stepping bit for bit;
    odd lengths flip the buffer parity and force a recapture."""
    w = synthetic.bump2d(128, 16, 0)
    a = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=_dtype(dtype))
    b = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=_dtype(dtype))
    a.set_state(torch.from_numpy(w.U0))
    b.set_state(torch.from_numpy(w.U0))
    for rep, k in enumerate([10, 10, 10, 7, 7, 10]):
        a.step_graph(k)
        b.step(k)
        _ = torch.ones(4096, device="cuda").sum().item()
        a.sync()
        b.sync()
        assert np.array_equal(a.U.cpu().numpy(), b.U.cpu().numpy()), rep
        assert a.time_index == b.time_index
    sa, sb = gpu_state(a), gpu_state(b)
    for k in range(2):
        assert np.array_equal(sa.Phi[k], sb.Phi[k]) and np.array_equal(sa.Psi[k], sb.Psi[k])
    a.close()
    b.close()



@pytest.mark.parametrize("multi", ["two", "three", "four", "five", "eight", "eight-ahead"])
@pytest.mark.parametrize("rows", [0, 5, (15 << 16) | 6])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["bump", "ragged", "onesided", "c2", "batch", "nolayer"])
def test_twostep_matches_single_steps_and_oracle(dtype, case, rows, multi):
    """Two (three, four) steps per pass over the layer-free core (temporal
    blocking) plus single steps on the frame: bit-identical to single steps,
    and the oracle agrees; step counts that are not a multiple end with a
    shorter pass and/or a single step.  rows = 5 makes the kernel's tiles end
    in a remainder of rows; frame form 15 takes the frame's steps in one
    fused launch."""
    MULTI, depth = {"two": (dp.VARIANT_TWOSTEP, 0), "three": (dp.VARIANT_THREESTEP, 0),
                    "four": (dp.VARIANT_FOURSTEP, 0), "five": (dp.VARIANT_DEEP, 5), "eight": (dp.VARIANT_DEEP, 8),
                    "eight-ahead": (dp.VARIANT_DEEP, 16 | 8)}[multi]
    rng = np.random.default_rng(17)
    c2 = None
    batch = 1
    if case == "bump":
        w = synthetic.bump2d(128, 16, 0)
        n, lo, hi, sig, U0 = w.n, w.lo, w.hi, w.sigma, w.U0
    elif case == "ragged":
        n, lo, hi = [611, 203], [5, 9], [13, 2]
        sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(2)]
        U0 = synthetic.white_noise_disk(n, lo, hi, 60.0, 0.25, rng)
    elif case == "onesided":
        n, lo, hi = [300, 190], [0, 12], [0, 0]
        sig = [None, synthetic.sigma_ramp(n[1], 12, 0, 2.0)]
        U0 = synthetic.gaussian_sum(n, lo, hi, 8, 2.0, 6.0, rng)
    elif case == "c2":
        n, lo, hi = [220, 170], [10, 10], [10, 10]
        sig = [synthetic.sigma_ramp(n[a], 10, 10, 2.0) for a in range(2)]
        c2 = synthetic.smooth_c2(n, lo, hi, 6, 10.0, 30.0, 0.5, 8, rng)
        U0 = synthetic.gaussian_sum(n, lo, hi, 10, 2.0, 6.0, rng)
    elif case == "nolayer":
        n, lo, hi = [130, 45], [0, 0], [0, 0]
        sig = [None, None]
        U0 = synthetic.gaussian_sum(n, lo, hi, 6, 2.0, 6.0, rng)
    else:
        batch = 3
        n, lo, hi = [150, 140], [8, 8], [8, 8]
        sig = [synthetic.sigma_ramp(n[a], 8, 8, 2.0) for a in range(2)]
        U0 = np.stack([synthetic.gaussian_sum(n, lo, hi, 5, 2.0, 6.0, rng) for _ in range(batch)])
    dt = 0.5 if c2 is None else 0.5 / math.sqrt(float(np.max(c2)))
    steps = 121
    print("case %s-step %s %s rows %d" % (multi, case, dtype, rows), flush=True)
    outs = []
    for variant in (MULTI, dp.VARIANT_CELL):
        sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=1.0 if c2 is None else c2, dtype=_dtype(dtype), batch=batch)
        sim.set_variant(variant, (depth << 20) | rows if variant == MULTI else 0)
        sim.set_state(torch.from_numpy(U0))
        sim.step(steps)
        sim.sync()
        outs.append((sim.U.cpu().numpy().copy(), sim.field(dp.FIELD_UPREV).cpu().numpy().copy(),
                     [sim.field(dp.FIELD_PHI(a)).cpu().numpy().copy() for a in range(2) if lo[a] + hi[a] > 0],
                     [sim.field(dp.FIELD_PSI(a)).cpu().numpy().copy() for a in range(2) if lo[a] + hi[a] > 0]))
        if variant == MULTI and batch == 1:
            gs = gpu_state(sim)
        sim.close()
    (a0, a1, a2, a3), (b0, b1, b2, b3) = outs
    assert np.array_equal(a0, b0) and np.array_equal(a1, b1)
    for x, y in zip(a2 + a3, b2 + b3):
        assert np.array_equal(x, y)
    if batch == 1:
        N = [lo[a] + n[a] + hi[a] for a in range(2)]
        g = oracle.Grid(N, 1.0, dt, sig, c2=c2)
        ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
        _assert_errs(compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant", [dp.VARIANT_TWOSTEP, dp.VARIANT_THREESTEP, dp.VARIANT_FOURSTEP,
                                     (dp.VARIANT_DEEP, 5), (dp.VARIANT_DEEP, 7), (dp.VARIANT_DEEP, 16 | 6)])
@pytest.mark.parametrize("group,rows", [(1, 3), (4, 7), (4, 4), (2, 1), (1 << 4 | 4, 8), (3 << 4 | 2, 5),
                                        (5 << 4 | 4, 6), (15 << 4 | 2, 6), (15 << 4 | 4, 17)])
def test_multistep_launch_shapes_bit_identical(dtype, variant, group, rows):
    """Every load-group size and tile height of the multi-step core kernels
    (2, 3, 4, 5 and 7 levels, and 6 with the loads issued a group ahead) (tiles shorter than a group, one-row tiles), and the frame's
    steps one thread per cell, as wave marches over spans of 1, 3 or 5 rows,
    or fused into one launch (group's high bits), give the single-step
    result bit for bit, with a c^2 field and a ragged grid."""
    rng = np.random.default_rng(5)
    n, lo, hi = [333, 157], [7, 11], [9, 4]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(2)]
    c2 = synthetic.smooth_c2(n, lo, hi, 6, 10.0, 30.0, 0.5, 8, rng)
    U0 = synthetic.gaussian_sum(n, lo, hi, 8, 2.0, 6.0, rng)
    dt = 0.5 / math.sqrt(float(np.max(c2)))
    depth = 0
    if isinstance(variant, tuple):
        variant, depth = variant
    outs = []
    for v, tr in ((variant, (depth << 20) | (group << 12) | rows), (dp.VARIANT_CELL, 0)):
        sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=c2, dtype=_dtype(dtype))
        sim.set_variant(v, tr)
        sim.set_state(torch.from_numpy(U0))
        sim.step(47)
        sim.sync()
        outs.append((sim.U.cpu().numpy().copy(), sim.field(dp.FIELD_UPREV).cpu().numpy().copy(),
                     [sim.field(dp.FIELD_PHI(a)).cpu().numpy().copy() for a in range(2)]))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    for x, y in zip(outs[0][2], outs[1][2]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("tile_rows", [0, (3 << 16) | (4 << 12) | 8, (15 << 16) | (4 << 12) | 8])
@pytest.mark.parametrize("variant", [dp.VARIANT_TWOSTEP, dp.VARIANT_THREESTEP, dp.VARIANT_FOURSTEP,
                                     (dp.VARIANT_DEEP, 6), (dp.VARIANT_DEEP, 8)])
def test_twostep_graph_replay_matches_eager(variant, tile_rows):
    if isinstance(variant, tuple):
        variant, depth = variant
        tile_rows |= depth << 20
    w = synthetic.bump2d(200, 20, 0)
    a = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    b = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float32)
    a.set_variant(variant, tile_rows)
    a.set_state(torch.from_numpy(w.U0))
    b.set_state(torch.from_numpy(w.U0))
    for rep, k in enumerate([10, 10, 7, 7, 10]):
        a.step_graph(k)
        b.step(k)
        _ = torch.ones(4096, device="cuda").sum().item()
        a.sync()
        b.sync()
        assert np.array_equal(a.U.cpu().numpy(), b.U.cpu().numpy()), rep
    a.close()
    b.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_launch_timing_counts_and_bytes(dtype):
    """The library's per-launch timing: one record per step-kernel launch,
    the algorithmic byte model per launch (3 words per cell, 4 per layer
    axis-cell; a pass's core launch 4 words per core cell), so that a pass of
    D levels stands for the bytes of D single steps; graph replays are not
    timed."""
    w = synthetic.bump2d(200, 20, 0)
    esize = 4 if dtype == "f32" else 8
    cells = w.N[0] * w.N[1]
    aux = sum((w.lo[a] + w.hi[a]) * (cells // w.N[a]) for a in range(2))
    step_bytes = (3 * cells + 4 * aux) * esize
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=_dtype(dtype))
    sim.set_state(torch.from_numpy(w.U0))
    sim.set_variant(dp.VARIANT_CELL, 0)
    sim.set_timing(True)
    sim.step(6)
    t = sim.get_timing()
    assert set(t) == {"step"} and t["step"]["launches"] == 6
    assert t["step"]["bytes"] == 6 * step_bytes and t["step"]["ms"] > 0
    # a pass of D levels: the core launch counts what it must move (4 words
    # per core cell), the frame's launches their steps' share; together they
    # stand for D steps: frame + (3 D / 4) core = D single steps
    sim.set_variant(dp.VARIANT_TWOSTEP, 0)
    sim.step(7)                                   # three pairs and one single step
    t = sim.get_timing()
    assert t["pair"]["launches"] == 3 and t["frame"]["launches"] == 3 * 2 and t["step"]["launches"] == 1
    assert t["frame"]["bytes"] + 1.5 * t["pair"]["bytes"] == pytest.approx(3 * 2 * step_bytes, rel=1e-12)
    assert t["step"]["bytes"] == step_bytes
    for variant, rows, steps, depth, frames in ((dp.VARIANT_THREESTEP, 0, 9, 3, 9), (dp.VARIANT_FOURSTEP, 0, 8, 4, 8),
                                                (dp.VARIANT_DEEP, 6 << 20, 12, 6, 12),
                                                (dp.VARIANT_DEEP, (6 << 20) | (15 << 16), 12, 6, 2)):
        sim.set_variant(variant, rows)
        sim.step(steps)
        t = sim.get_timing()
        assert t["pair"]["launches"] == steps // depth and t["frame"]["launches"] == frames and "step" not in t
        assert t["frame"]["bytes"] + 0.75 * depth * t["pair"]["bytes"] == pytest.approx(steps * step_bytes, rel=1e-12)
    sim.set_variant(dp.VARIANT_FOURSTEP, 0)
    sim.step(11)                                  # two quadruples and one triple
    t = sim.get_timing()
    assert t["pair"]["launches"] == 3 and t["frame"]["launches"] == 2 * 4 + 3 and "step" not in t
    sim.step_graph(4)
    sim.sync()
    assert sim.get_timing() == {}
    sim.set_timing(False)
    sim.step(2)
    assert sim.get_timing() == {}
    sim.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ndim,variant,tile_rows,walls,lo,hi", [
    (2, dp.VARIANT_TWOSTEP, 0, (True, True), [7, 12], [10, 5]),
    (2, dp.VARIANT_THREESTEP, 0, (True, False), [0, 12], [10, 5]),
    (2, dp.VARIANT_THREESTEP, (3 << 16) | (4 << 12) | 8, (False, True), [7, 12], [10, 1]),
    (2, dp.VARIANT_THREESTEP, 0, (True, True), [7, 12], [10, 0]),       # no layer cell above: single steps
    (2, dp.VARIANT_FOURSTEP, 0, (True, True), [7, 12], [10, 5]),
    (2, dp.VARIANT_FOURSTEP, (2 << 16) | (2 << 12) | 6, (False, True), [7, 12], [10, 1]),
    (2, dp.VARIANT_DEEP, (8 << 20) | (4 << 12) | 12, (True, True), [9, 12], [10, 1]),
    (2, dp.VARIANT_DEEP, (8 << 20) | (15 << 16) | (4 << 12) | 12, (True, True), [9, 12], [10, 1]),
    (2, dp.VARIANT_THREESTEP, (15 << 16) | 8, (True, False), [0, 12], [10, 5]),
    (3, dp.VARIANT_TWOSTEP, 0, (True, False, True), [5, 3, 6], [4, 7, 5]),
    (3, dp.VARIANT_TWOSTEP, 0, (True, True, True), [0, 3, 6], [4, 7, 1]),
    # the marching frames (bits 19 and 30) are for periodic axes: with walls the frame's single steps
    # take the box kernels
    (3, dp.VARIANT_TWOSTEP, (1 << 30) | (1 << 29) | (1 << 19) | (8 << 12) | 16, (True, False, True), [5, 3, 6],
     [4, 7, 5]),
    (3, dp.VARIANT_TWOSTEP, (1 << 28) | (1 << 19) | (8 << 20) | (8 << 12) | 16, (False, True, False), [5, 3, 6],
     [4, 7, 5]),
])
def test_multistep_with_walls_bit_identical_and_oracle(dtype, ndim, variant, tile_rows, walls, lo, hi):
    """Multi-step passes on grids truncated by reflecting walls: the cores read
    only cells inside the grid (every walled axis has a layer with a cell
    above the interior; otherwise the run takes single steps) and the frames
    step with the ghost cells at zero.  Bit for bit against single steps, and
    the oracle agrees, long enough for the wall echo to return."""
    rng = np.random.default_rng(45)
    if ndim == 2:
        n, steps, dt = [170, 121], 161, 0.5
    else:
        n, steps, dt = [34, 27, 23], 61, 0.4
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(ndim)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 6, 2.0, 6.0, rng)
    N = [lo[a] + n[a] + hi[a] for a in range(ndim)]
    print("case multistep walls=%s %dD %s variant=%d lo=%s hi=%s" % (walls, ndim, dtype, variant, lo, hi), flush=True)
    outs = []
    for v, tr in ((variant, tile_rows), (dp.VARIANT_CELL, 0)):
        sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, dtype=_dtype(dtype), walls=walls)
        sim.set_variant(v, tr)
        sim.set_state(torch.from_numpy(U0))
        sim.step(steps)
        sim.sync()
        outs.append([sim.U.cpu().numpy().copy(), sim.field(dp.FIELD_UPREV).cpu().numpy().copy()]
                    + [sim.field(f(a)).cpu().numpy().copy() for a in range(ndim) for f in (dp.FIELD_PHI, dp.FIELD_PSI)])
        if v == variant:
            gs = gpu_state(sim)
        sim.close()
    for k, (x, y) in enumerate(zip(outs[0], outs[1])):
        assert np.array_equal(x, y), k
    g = oracle.Grid(N, 1.0, dt, sig, walls=walls)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
    _assert_errs(compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None), dtype)
