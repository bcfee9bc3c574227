"""The paper's central claim on the GPU path (Thm. 1; Sec. 1.1.3, Figs. 2
and 3): a run truncated by the discrete layer equals, on the physical domain,
the plain discrete wave equation on a domain so large that no wave reaches
its edge (the oracle's free-space run, periodic with a margin of at least
steps + 1 cells: the leapfrog light cone grows one cell per step).

Two readings bound what "equals" means (both measured on the oracle and
kept in the design notes):
  * the initial data must start in the physical domain away from the layer:
    data on the interior cells next to an interface (the first two on the low
    side, the last on the high side) does not continue into the layer as a
    free-space wave and differs by O(1e-3) of the peak from the first step;
    with those cells zero the difference is rounding (2e-16);
  * the band is periodic: after waves have crossed it (64 cells here, so no
    earlier than step 65) the difference also holds the residual waves the
    layer has not absorbed (high-frequency and grazing content; Fig. 5c: they
    fall exponentially with the layer's thickness), which grow with time.
So the exact claim is checked before the first crossing, and the residual
after the workload's full run is recorded (the oracle's own truncated run
shows the same growth at 1088^2: 2e-16 of the initial peak at step 64,
3e-12 at 250, 9e-8 at 500, 6e-5 at 1000) against a loose bound that only
says the layer absorbs and the run stays stable.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


def _tuned(w, dtype):
    from paper_1804_01390_amd import autotune
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_state(torch.from_numpy(w.U0))
    autotune.tune(sim)                      # the launch the benchmark times (cached per grid)
    sim.set_state(torch.from_numpy(w.U0))
    return sim


def _free_space(w, Nr, steps_list):
    """The oracle's plain wave equation on an Nr^2 periodic grid with the
    workload's interior data centred in it; yields (steps, U interior)."""
    n, m = w.n[0], w.lo[0]
    off = (Nr - n) // 2
    U0 = np.zeros((Nr, Nr))
    U0[off:off + n, off:off + n] = w.U0[m:m + n, m:m + n]
    g = oracle.Grid([Nr, Nr], w.h, w.dt, [None, None])
    s = oracle.start(g, U0)
    U, Up, done = s.U, s.Uprev, 0
    for t in steps_list:
        U, Up = oracle.wave_run(g, U, Up, t - done)
        done = t
        yield t, U[off:off + n, off:off + n]


def test_c1_bump_matches_free_space_fp64():
    """128^2 + 16-cell layer, Gaussian bump of width 4 at the centre, 500
    steps, FP64, in the tuned launch; free space on 640^2."""
    w = synthetic.bump2d(128, 16, 500)
    print("case reflection c1 160^2 fp64 500 steps vs 640^2", flush=True)
    sim = _tuned(w, torch.float64)
    sim.step(w.steps)
    got = sim.U.cpu().numpy()[16:144, 16:144]
    sim.close()
    (_, ref), = list(_free_space(w, 640, [w.steps]))
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(w.U0)))
    print("c1: max|U - U_free| / max|U0| = %.3e after %d steps" % (err, w.steps), flush=True)
    assert err <= 1e-11


@pytest.fixture(scope="module")
def c2_reference():
    """Config 2's interior data (64 seeded bumps on 4096^2, the two cells next
    to each interface zeroed) and its free-space run on 6144^2 at steps 64
    and 2000."""
    w = synthetic.bumps2d(n=4096, m=32, steps=2000, seed=0, margin=2)
    print("case reflection c2: oracle free space 6144^2, 2000 steps", flush=True)
    refs = dict((t, u.copy()) for t, u in _free_space(w, 6144, [64, 2000]))
    return w, refs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_bumps_match_free_space(dtype, c2_reference):
    """4096^2 + 32-cell layer, the tuned launch; after 64 steps (no wave can
    have crossed the 64-cell band) the truncated run equals free space to
    rounding: FP64 <= 1e-13, FP32 <= 2e-5 of the initial peak.  After the
    workload's 2000 steps the difference is the layer's residual (recorded;
    below 1e-2 of the initial peak)."""
    w, refs = c2_reference
    td = torch.float64 if dtype == "f64" else torch.float32
    print("case reflection c2 %s" % dtype, flush=True)
    sim = _tuned(w, td)
    peak = float(np.max(np.abs(w.U0)))
    out = {}
    done = 0
    for t in (64, 2000):
        sim.step(t - done)
        done = t
        got = sim.U.double().cpu().numpy()[32:4128, 32:4128]
        out[t] = float(np.max(np.abs(got - refs[t])) / peak)
        print("c2 %s: max|U - U_free| / max|U0| = %.3e after %d steps" % (dtype, out[t], t), flush=True)
    sim.close()
    assert out[64] <= (1e-13 if dtype == "f64" else 2e-5)
    assert out[2000] <= 1e-2
