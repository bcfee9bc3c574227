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


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_tuner_candidate_is_bit_identical(dtype):
    """Each launch shape the tuner may pick for a 2D grid (multi-step passes
    of 2 to 8 levels, every frame form, loads issued ahead) gives the fields
    of one-thread-per-cell single steps bit for bit, over a step count that
    ends in shorter passes."""
    from paper_1804_01390_amd import autotune
    w = synthetic.bumps2d(n=300, m=16, steps=0, seed=4)
    steps = 37
    outs = {}
    for variant, tr in [(dp.VARIANT_CELL, 0)] + list(autotune.CANDIDATES_2D):
        sim = dp.Simulation(w.n, w.lo, w.hi, w.h, w.dt, w.sigma, dtype=dtype)
        sim.set_variant(variant, tr)
        sim.set_state(torch.from_numpy(w.U0))
        sim.step(steps)
        sim.sync()
        outs[(variant, tr)] = (sim.U.cpu().numpy().copy(), sim.field(dp.FIELD_UPREV).cpu().numpy().copy(),
                               sim.field(dp.FIELD_PHI(1)).cpu().numpy().copy())
        sim.close()
    ref = outs[(dp.VARIANT_CELL, 0)]
    for key, o in outs.items():
        for a, b in zip(ref, o):
            assert np.array_equal(a, b), key


def test_every_problem_set_candidate_is_bit_identical():
    """Each (variant, rows, group) the problem-set tuner may pick gives the
    same fields as single steps, eagerly and from a captured graph."""
    from paper_1804_01390_amd import autotune
    probs = [synthetic.bump2d(s, m, 0, 2.0, 2.0, 1.0, 0.5) for s, m in [(96, 16), (150, 20), (64, 17)]]
    outs = {}
    for variant, rows, group in [(dp.VARIANT_MARCH, 32, 4)] + list(autotune.CANDIDATES_MULTI):
        sim = dp.MultiSimulation(probs, dtype=torch.float32)
        sim.set_variant(variant, rows, group)
        sim.set_state([w.U0 for w in probs])
        sim.step(19, graph=True)
        sim.step(12)
        sim.sync()
        outs[(variant, rows, group)] = [sim.field(i, f).cpu().numpy().copy() for i in range(len(probs))
                                        for f in (dp.FIELD_U, dp.FIELD_UPREV)]
        sim.close()
    ref = outs[(dp.VARIANT_MARCH, 32, 4)]
    for key, o in outs.items():
        for a, b in zip(ref, o):
            assert np.array_equal(a, b), key
