"""Multi-step 2D passes with point sources and receivers (the adjoint
workload's shots and traces; not part of the paper).  The deep cores add the
sources at every level they form and record the receivers lying deep enough
in the core; the frame's per-step launches record the rest.  Every field and
every trace must equal single steps (one thread per cell) bit for bit, and
the traces the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
import synthetic
from helpers import rel_err

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


def _setup(batch, c2field):
    """2D 150x130 interior + 12/9-cell layers, a Ricker source per member
    inside the core, receivers on a whole interior row (crossing from the
    frame into the core) plus a few scattered near the layer."""
    rng = np.random.default_rng(12)
    n, lo, hi = [150, 130], [12, 9], [10, 11]
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    cells = N[0] * N[1]
    sig = [synthetic.sigma_ramp(n[a], lo[a], hi[a], 2.0) for a in range(2)]
    c2 = synthetic.smooth_c2(n, lo, hi, 4, 10.0, 30.0, 0.4, 3, rng) if c2field else None
    dt = 0.5 / math.sqrt(1.4) if c2field else 0.5
    steps = 61
    src_local = [synthetic.flat_index(N, [lo[0] + 30 + 17 * b, lo[1] + 40]) for b in range(batch)]
    sources = [b * cells + src_local[b] for b in range(batch)]
    f = 1.0 / 10.0
    wav = np.stack([synthetic.ricker(steps, dt, f, 1.5 / f) * (1.0 + 0.3 * b) for b in range(batch)])
    row = lo[1] + 50
    rec_local = [synthetic.flat_index(N, [x, row]) for x in range(lo[0], lo[0] + n[0])]
    rec_local += [synthetic.flat_index(N, p) for p in ([lo[0], lo[1]], [lo[0] + 3, lo[1] + 100],
                                                        [lo[0] + n[0] - 1, lo[1] + 7], [lo[0] + 70, lo[1] + n[1] - 2],
                                                        [lo[0] + 71, lo[1] + 64])]
    receivers = [b * cells + r for b in range(batch) for r in rec_local]
    return dict(n=n, lo=lo, hi=hi, N=N, sig=sig, c2=c2, dt=dt, steps=steps, sources=sources, wav=wav,
                receivers=receivers, src_local=src_local, rec_local=rec_local, batch=batch)


def _run(cfg, dtype, variant, tile_rows, timing=False, walls=()):
    td = torch.float64 if dtype == "f64" else torch.float32
    sim = dp.Simulation(cfg["n"], cfg["lo"], cfg["hi"], 1.0, cfg["dt"], cfg["sig"],
                        c2=1.0 if cfg["c2"] is None else cfg["c2"], dtype=td, batch=cfg["batch"], walls=walls)
    sim.set_variant(variant, tile_rows)
    sim.set_state(torch.zeros(sim.shape, dtype=td, device="cuda"))
    sim.inject(cfg["sources"], torch.from_numpy(cfg["wav"]).to(td))
    tr = sim.record(cfg["receivers"], cfg["steps"])
    if timing:
        sim.set_timing(True)
    sim.step(cfg["steps"])
    sim.sync()
    t = sim.get_timing() if timing else None
    fields = [sim.field(dp.FIELD_U).cpu().numpy(), sim.field(dp.FIELD_UPREV).cpu().numpy()]
    for a in range(2):
        fields += [sim.field(dp.FIELD_PHI(a)).cpu().numpy(), sim.field(dp.FIELD_PSI(a)).cpu().numpy()]
    out = tr.cpu().numpy().copy()
    sim.close()
    return out, fields, t


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant,tile_rows", [(dp.VARIANT_DEEP, 4 << 20), (dp.VARIANT_DEEP, (8 << 20) | 32),
                                               (dp.VARIANT_DEEP, (1 << 24) | (6 << 20) | (4 << 12) | 16),
                                               (dp.VARIANT_FOURSTEP, 7),
                                               (dp.VARIANT_DEEP, (5 << 20) | (3 << 16) | 24)])
@pytest.mark.parametrize("batch,c2field", [(1, False), (3, True)])
def test_passes_with_sources_and_receivers_bit_identical(dtype, variant, tile_rows, batch, c2field):
    cfg = _setup(batch, c2field)
    print("case taps2d %s variant=%d rows=0x%x batch=%d c2=%s" % (dtype, variant, tile_rows, batch, c2field),
          flush=True)
    ref_tr, ref_f, _ = _run(cfg, dtype, dp.VARIANT_CELL, 0)
    got_tr, got_f, t = _run(cfg, dtype, variant, tile_rows, timing=True)
    assert t["pair"]["launches"] >= 7                       # the run went as multi-step passes
    assert np.array_equal(got_tr, ref_tr)
    for a, b in zip(got_f, ref_f):
        assert np.array_equal(a, b)


def test_pass_traces_match_oracle():
    """FP64 traces of a deep-pass run against the oracle (member 0 and 2 of a
    3-member batch with a c^2 field)."""
    cfg = _setup(3, True)
    tr, _, _ = _run(cfg, "f64", dp.VARIANT_DEEP, 8 << 20)
    nrec = len(cfg["rec_local"])
    for b in (0, 2):
        g = oracle.Grid(cfg["N"], 1.0, cfg["dt"], cfg["sig"], c2=cfg["c2"])
        s0 = oracle.start(g, np.zeros(tuple(reversed(cfg["N"]))))
        _, rtr = oracle.run(g, s0, cfg["steps"], sources=[cfg["src_local"][b]], wavelets=cfg["wav"][b:b + 1],
                            receivers=cfg["rec_local"], nt=cfg["steps"])
        err = rel_err(tr[b * nrec:(b + 1) * nrec], rtr)
        print("member %d traces err %.2e" % (b, err), flush=True)
        assert err <= 1e-12


def test_source_outside_the_shrunk_core_takes_single_steps():
    """A source less than levels-1 cells inside the core: the run falls back
    to shallower passes or single steps and stays bit-identical."""
    cfg = _setup(1, False)
    N = cfg["N"]
    cfg["sources"] = [synthetic.flat_index(N, [cfg["lo"][0] + 3, cfg["lo"][1] + 40])]
    ref_tr, ref_f, _ = _run(cfg, "f64", dp.VARIANT_CELL, 0)
    got_tr, got_f, t = _run(cfg, "f64", dp.VARIANT_DEEP, 8 << 20, timing=True)
    assert "pair" not in t
    assert np.array_equal(got_tr, ref_tr)
    for a, b in zip(got_f, ref_f):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_passes_with_taps_inside_reflecting_walls(dtype):
    """The same with both axes walled (each has a layer cell above the
    interior, so the passes apply): bit for bit against single steps."""
    cfg = _setup(2, True)
    print("case taps2d walls %s" % dtype, flush=True)
    ref_tr, ref_f, _ = _run(cfg, dtype, dp.VARIANT_CELL, 0, walls=(True, True))
    for variant, tile_rows in ((dp.VARIANT_DEEP, 8 << 20), (dp.VARIANT_DEEP, (5 << 20) | (4 << 12) | 16)):
        got_tr, got_f, t = _run(cfg, dtype, variant, tile_rows, timing=True, walls=(True, True))
        assert t["pair"]["launches"] >= 7
        assert np.array_equal(got_tr, ref_tr)
        for a, b in zip(got_f, ref_f):
            assert np.array_equal(a, b)
