"""The tile-shape autotuner picks a launch shape without changing results."""
import os

import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_autotune_choice_is_bit_identical(tmp_path, dtype):
    from paper_1804_01390_amd import autotune
    w = synthetic.bumps2d(n=900, m=20, steps=0, seed=2)
    sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    sim.set_state(torch.from_numpy(w.U0))
    cache = str(tmp_path / "cache.json")
    rec = autotune.tune(sim, steps=5, cache=cache)
    assert not rec["cached"] and len(rec["timings"]) >= 5
    assert sim.time_index == 0
    rec2 = autotune.tune(sim, steps=5, cache=cache)
    assert rec2["cached"] and rec2["tile_rows"] == rec["tile_rows"]
    sim.step(40)
    sim.sync()
    tuned = sim.U.cpu().numpy().copy()
    ref = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
    ref.set_variant(dp.VARIANT_CELL, 0)
    ref.set_state(torch.from_numpy(w.U0))
    ref.step(40)
    ref.sync()
    assert np.array_equal(tuned, ref.U.cpu().numpy())
    sim.close()
    ref.close()
