"""The entry point that allocates nothing (dpml_step_checked_noalloc: the
non-finite watchdog's flags in the library's static device array, steps by
one thread per cell) against dpml_step_checked on the same inputs, bit for
bit, on two calls in a row, the second with a smaller grid; and the same
non-finite report when a NaN is in the initial field."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


def _arrays(sim):
    out = [sim.field(dp.FIELD_U).cpu().numpy(), sim.field(dp.FIELD_UPREV).cpu().numpy()]
    for a in range(sim.ndim):
        if sim.lo[a] + sim.hi[a]:
            out += [sim.field(dp.FIELD_PHI(a)).cpu().numpy(), sim.field(dp.FIELD_PSI(a)).cpu().numpy()]
    return out


def _pair(w, dtype, U0, variant):
    sims = []
    for _ in range(2):
        s = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
        s.set_variant(*variant)
        s.set_state(torch.from_numpy(U0))
        sims.append(s)
    return sims


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_checked_on_two_calls(dtype):
    # a 3D grid stepped as multi-step passes by the checked entry point, then a
    # smaller 2D grid; each against the allocation-free entry point
    big = synthetic.ricker3d(n=60, m=6, steps=40, ppw=8.0)
    big.U0 = synthetic.gaussian_sum(big.n, big.lo, big.hi, 4, 2.0, 5.0, np.random.default_rng(2))
    small = synthetic.bump2d((70, 41), 7, 0)
    for w, variant, steps, every in ((big, (dp.VARIANT_TWOSTEP, 0), 23, 5), (small, (dp.VARIANT_DEEP, 6 << 20), 17, 4)):
        print("case noalloc %s %dD cells=%d" % (dtype, w.ndim, w.cells), flush=True)
        ref, new = _pair(w, dtype, w.U0, variant)
        ref.step_checked(steps, every)
        new.step_checked_noalloc(steps, every)
        assert new.time_index == ref.time_index == steps
        for a, b in zip(_arrays(new), _arrays(ref)):
            assert np.array_equal(a, b)
        ref.close()
        new.close()


def test_noalloc_reports_nonfinite_like_checked():
    w = synthetic.bump2d(64, 8, 0)
    U0 = w.U0.copy()
    U0[40, 40] = np.nan
    codes = []
    for entry in ("step_checked", "step_checked_noalloc"):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=torch.float64)
        sim.set_state(torch.from_numpy(U0))
        with pytest.raises(dp.DpmlError) as ei:
            getattr(sim, entry)(20, 5)
        codes.append((ei.value.code, sim.time_index))
        sim.close()
    assert codes[0] == codes[1] == (dp.DPML_ENONFINITE, 5)
