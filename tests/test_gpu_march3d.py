"""The 3D register-neighbour marching step (variant MARCH in 3D: k_march3d
over a layer-free core box and the x-band, z-band and y-band boxes) against
one thread per cell (bit for bit: both evaluate the scheme in the same
operation order) and against the FP64 oracle, over its launch shapes (rows
per wave, planes of loads in flight, planes per chunk) and the layer
geometries that change its code paths: ragged extents, layers of one side
only, an axis without a layer, one-cell layers, layers wider than a strip's
outputs, batches and a c^2 field."""
import math

import numpy as np
import pytest

import oracle
import synthetic
from helpers import compare_states, gpu_state, run_with_peaks

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


def march_shape(chunk=0, ry=0, ryl=1, core_first=False, split=False, lchunk=0):
    """tile_rows of a 3D MARCH launch: planes per core chunk (bits 0-11), rows
    per core wave (bits 12-15: 1, 2, 4 or 8), rows per wave of the z- and
    x-band boxes (bits 16-17: 1, 2 or 4), the core's waves first (bit 18),
    core and layer boxes as two launches (bit 19), planes per layer chunk
    (bits 20-27)."""
    return (chunk | (ry << 12) | ({1: 0, 2: 1, 4: 2}[ryl] << 16) | (int(core_first) << 18) | (int(split) << 19)
            | (lchunk << 20))


SHAPES = [march_shape(), march_shape(5, 4, 2, lchunk=3), march_shape(7, 8, 4, core_first=True),
          march_shape(64, 2, 1, split=True), march_shape(3, 1, 2, core_first=True, split=True, lchunk=200),
          march_shape(9, 2, 4, lchunk=5)]


def _case(name, rng):
    if name == "ragged":
        n, lo, hi = [45, 38, 33], [6, 3, 7], [4, 8, 5]
    elif name == "onesided":
        n, lo, hi = [70, 21, 19], [0, 5, 4], [6, 0, 3]
    elif name == "nolayer_x":
        n, lo, hi = [40, 30, 26], [0, 4, 3], [0, 5, 6]
    elif name == "thin":
        n, lo, hi = [66, 17, 15], [1, 1, 0], [0, 1, 1]
    elif name == "wide_layer":
        n, lo, hi = [20, 16, 14], [40, 9, 6], [33, 8, 7]   # the x band spans more than one strip
    else:
        raise ValueError(name)
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) if lo[a] + hi[a] else None for a in range(3)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 6, 2.0, 5.0, rng)
    return n, lo, hi, sig, U0


def _state_arrays(sim):
    out = [sim.field(dp.FIELD_U).cpu().numpy(), sim.field(dp.FIELD_UPREV).cpu().numpy()]
    for a in range(3):
        if sim.lo[a] + sim.hi[a]:
            out += [sim.field(dp.FIELD_PHI(a)).cpu().numpy(), sim.field(dp.FIELD_PSI(a)).cpu().numpy()]
    return out


def _run(n, lo, hi, sig, U0, steps, dtype, variant, tile_rows, batch=1, c2=1.0, dt=0.4):
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=c2, dtype=dtype, batch=batch)
    sim.set_variant(variant, tile_rows)
    U = torch.from_numpy(U0)
    if batch > 1:
        U = torch.stack([U * (1.0 + 0.25 * b) for b in range(batch)])
    sim.set_state(U)
    sim.step(steps)
    sim.sync()
    return sim


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", ["ragged", "onesided", "nolayer_x", "thin", "wide_layer"])
@pytest.mark.parametrize("shape", SHAPES)
def test_march3d_bit_identical_to_cells_and_oracle(dtype, case, shape):
    rng = np.random.default_rng(31)
    n, lo, hi, sig, U0 = _case(case, rng)
    td = torch.float64 if dtype == "f64" else torch.float32
    steps = 23
    print("case march3d %s %s shape=0x%x" % (case, dtype, shape), flush=True)
    ref_sim = _run(n, lo, hi, sig, U0, steps, td, dp.VARIANT_CELL, 0)
    want = _state_arrays(ref_sim)
    ref_sim.close()
    sim = _run(n, lo, hi, sig, U0, steps, td, dp.VARIANT_MARCH, shape)
    got = _state_arrays(sim)
    for k, (a, b) in enumerate(zip(got, want)):
        assert np.array_equal(a, b), "field %d differs from one thread per cell" % k
    gs = gpu_state(sim)
    sim.close()
    N = [lo[a] + n[a] + hi[a] for a in range(3)]
    g = oracle.Grid(N, 1.0, 0.4, sig)
    ref, _, peaks = run_with_peaks(g, oracle.start(g, U0), steps, n, lo, hi)
    errs = compare_states(gs, ref, n, lo, hi, peaks if dtype == "f32" else None)
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= TOL[dtype], (k, v)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_march3d_batch_and_c2_field(dtype):
    """Two batch members, and (separately) a per-cell c^2: each bit for bit
    against one thread per cell."""
    rng = np.random.default_rng(7)
    n, lo, hi = [52, 27, 24], [5, 4, 3], [3, 5, 6]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(3)]
    U0 = synthetic.gaussian_sum(n, lo, hi, 5, 2.0, 5.0, rng)
    td = torch.float64 if dtype == "f64" else torch.float32
    print("case march3d batch %s" % dtype, flush=True)
    for kw in ({"batch": 2}, {"c2": synthetic.smooth_c2(n, lo, hi, 4, 6.0, 12.0, 0.4, 2, rng),
                              "dt": 0.4 / math.sqrt(1.4)}):
        outs = []
        for variant, tr in ((dp.VARIANT_CELL, 0), (dp.VARIANT_MARCH, march_shape(9, 8, 2)),
                            (dp.VARIANT_MARCH, march_shape(0, 4, 4, core_first=True))):
            sim = _run(n, lo, hi, sig, U0, 17, td, variant, tr, **kw)
            outs.append(_state_arrays(sim))
            sim.close()
        for other in outs[1:]:
            for a, b in zip(other, outs[0]):
                assert np.array_equal(a, b)
