"""Edge cases of the stepping paths: zero steps, grids too small for the
multi-step passes (they fall back to single steps), one-cell layers, problem
sets that mix problems with and without a multi-step core, and a layer with
zero damping.  Every case is checked bit for bit against single steps and
against the oracle."""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import compare_states, gpu_state, run_with_peaks

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu

# (variant, tile_rows)
VARIANTS = [(dp.VARIANT_CELL, 0), (dp.VARIANT_MARCH, 0), (dp.VARIANT_MARCH1, 0), (dp.VARIANT_TWOSTEP, 0),
            (dp.VARIANT_THREESTEP, 0), (dp.VARIANT_FOURSTEP, 0), (dp.VARIANT_DEEP, 0), (dp.VARIANT_DEEP, 8 << 20),
            (dp.VARIANT_TWOSTEP, 15 << 16), (dp.VARIANT_DEEP, (8 << 20) | (15 << 16))]


def _fields(sim, ndim):
    return ([sim.U.cpu().numpy().copy(), sim.field(dp.FIELD_UPREV).cpu().numpy().copy()]
            + [sim.field(f(a)).cpu().numpy().copy() for a in range(ndim) for f in (dp.FIELD_PHI, dp.FIELD_PSI)
               if sim.lo[a] + sim.hi[a] > 0])


@pytest.mark.parametrize("variant,tile_rows", VARIANTS)
def test_zero_steps_change_nothing(variant, tile_rows):
    w = synthetic.bump2d(40, 6, 0)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
    sim.set_variant(variant, tile_rows)
    sim.set_state(torch.from_numpy(w.U0))
    sim.step(7)
    sim.sync()
    before = _fields(sim, 2)
    t0 = sim.time_index
    sim.step(0)
    sim.step_graph(0)
    sim.sync()
    for a, b in zip(before, _fields(sim, 2)):
        assert np.array_equal(a, b)
    assert sim.time_index == t0
    sim.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("ndim,n,lo,hi", [
    (2, [5, 6], [1, 1], [1, 1]),          # extents below 8: single steps only
    (2, [11, 9], [1, 1], [1, 1]),         # one-cell layers: tiny cores
    (2, [3, 40], [2, 0], [2, 0]),         # no three-step core along x
    (3, [9, 10, 4], [1, 1, 1], [1, 1, 1]),  # z extent below 8
    (3, [12, 11, 13], [1, 2, 1], [2, 1, 1]),
])
def test_small_grids_and_thin_layers(dtype, ndim, n, lo, hi):
    rng = np.random.default_rng(31)
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(ndim)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 3, 1.0, 2.0, rng)
    N = [lo[a] + n[a] + hi[a] for a in range(ndim)]
    dt = 0.5 if ndim == 2 else 0.4
    steps = 37
    print("case small %dD n=%s lo=%s hi=%s %s" % (ndim, n, lo, hi, dtype), flush=True)
    outs = []
    for v, tr in VARIANTS:
        sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, dtype=dtype)
        sim.set_variant(v, tr)
        sim.set_state(torch.from_numpy(U0))
        sim.step(steps)
        sim.sync()
        outs.append(_fields(sim, ndim))
        if v == dp.VARIANT_CELL:
            gs = gpu_state(sim)
        sim.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    g = oracle.Grid(N, 1.0, dt, sig)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
    errs = compare_states(gs, ref, n, lo, hi, peaks if dtype == torch.float32 else None)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("variant,rows", [(dp.VARIANT_TWOSTEP, 0), (dp.VARIANT_THREESTEP, 0),
                                          (dp.VARIANT_FOURSTEP, 0), (dp.VARIANT_DEEP, 8 << 20)])
def test_problem_set_with_a_problem_too_small_for_passes(variant, rows):
    """One problem too small for a multi-step core makes the whole set take
    single steps (or two-step passes); the result does not change."""
    probs = [synthetic.bump2d(s, m, 0, 2.0, 2.0, 1.0, 0.5) for s, m in [(64, 8), (3, 2), (100, 12)]]
    outs = []
    for v in (variant, dp.VARIANT_MARCH):
        sim = dp.MultiSimulation(probs, dtype=torch.float64)
        sim.set_variant(v, rows if v == variant else 0, 0)
        sim.set_state([w.U0 for w in probs])
        sim.step(23, graph=True)
        sim.step(10)
        sim.sync()
        outs.append([sim.field(i, dp.FIELD_U).cpu().numpy().copy() for i in range(len(probs))])
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    for i, w in enumerate(probs):
        g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
        ref, _ = oracle.run(g, oracle.start(g, w.U0), 33)
        peak = max(float(np.max(np.abs(ref.U))), 1e-300)
        assert float(np.max(np.abs(outs[0][i] - ref.U))) / peak <= 1e-12


def test_layer_without_damping_is_the_plain_wave_equation():
    """sigma = 0 on a 16-cell band: Phi and Psi still integrate the gradient of
    U but no longer act on it, so every variant steps the plain leapfrog wave
    equation of the periodic grid; the auxiliary fields match the oracle run
    with the same zero profiles."""
    n, lo, hi = [90, 70], [16, 16], [16, 16]
    sig = [np.zeros(n[a] + lo[a] + hi[a]) for a in range(2)]
    rng = np.random.default_rng(2)
    U0 = synthetic.gaussian_sum(n, lo, hi, 4, 2.0, 5.0, rng)
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    g0 = oracle.Grid(N, 1.0, 0.5, [None, None])
    plain, _ = oracle.run(g0, oracle.start(g0, U0), 40)
    g = oracle.Grid(N, 1.0, 0.5, sig)
    ref, _ = oracle.run(g, oracle.start(g, U0), 40)
    for v, tr in VARIANTS:
        sim = dp.Simulation(n, lo, hi, 1.0, 0.5, sig, dtype=torch.float64)
        sim.set_variant(v, tr)
        sim.set_state(torch.from_numpy(U0))
        sim.step(40)
        sim.sync()
        assert float(np.max(np.abs(sim.U.cpu().numpy() - plain.U))) <= 1e-12 * float(np.max(np.abs(plain.U)))
        errs = compare_states(gpu_state(sim), ref, n, lo, hi)
        assert max(errs.values()) <= 1e-12, errs
        sim.close()
