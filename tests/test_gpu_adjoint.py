"""GPU adjoint parity: the library's checkpointed reverse-time adjoint
(through the C ABI) against the oracle's plain discrete adjoint, and the
torch.autograd interface against the same."""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-5}


def _shots(ndim=2, batch=3, steps=70, seed=0, wide=False, nolayer_x=False):
    rng = np.random.default_rng(seed)
    if ndim == 2 and nolayer_x:
        n, lo, hi = [130, 30], [0, 5], [0, 6]   # x periodic with no layer: the cores span it
    elif ndim == 2 and wide:
        n, lo, hi = [150, 27], [6, 5], [7, 6]   # several 64-column strips, ragged row groups
    elif ndim == 2:
        n, lo, hi = [40, 34], [6, 5], [7, 6]
    else:
        n, lo, hi = [18, 16, 14], [4, 3, 5], [5, 4, 3]
    N = [lo[a] + n[a] + hi[a] for a in range(ndim)]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) if lo[a] + hi[a] else None for a in range(ndim)]
    c2 = synthetic.smooth_c2(n, lo, hi, 4, 3.0, 6.0, 0.4, 2, rng)
    dt = 0.4 if ndim == 2 else 0.3
    srcs = []
    for b in range(batch):
        p = [lo[a] + 3 + (5 * b + 2 * a) % (n[a] - 6) for a in range(ndim)]
        srcs.append([synthetic.flat_index(N, p)])
    rec = [synthetic.flat_index(N, [lo[0] + x] + [lo[a] + n[a] - 4 for a in range(1, ndim)])
           for x in range(1, n[0] - 1, 3)]
    rec.append(srcs[0][0])
    rec.append(synthetic.flat_index(N, [1] * ndim))      # inside the layer
    wav = np.vstack([synthetic.ricker(steps, dt, 0.1 + 0.01 * b, 9.0 + b) for b in range(batch)])
    obs = rng.normal(scale=1e-3, size=(batch, len(rec), steps))
    return n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps


def _oracle_grads(n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps):
    g = oracle.Grid(N, 1.0, dt, sig, c2=c2)
    gc2 = np.zeros(tuple(reversed(N)))
    gw = np.zeros_like(wav)
    traces = []
    for b in range(len(srcs)):
        _, tr = oracle.run(g, oracle.start(g, np.zeros(tuple(reversed(N)))), steps, sources=srcs[b],
                           wavelets=wav[b:b + 1], receivers=rec, nt=steps)
        traces.append(tr)
        gcb, gwb = oracle.adjoint(g, np.zeros(tuple(reversed(N))), steps, srcs[b], wav[b:b + 1], rec,
                                  tr - obs[b])
        gc2 += gcb
        gw[b] = gwb[0]
    return gc2, gw, np.stack(traces)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("dtype,ndim,every,wide", [("f64", 2, 7, False), ("f32", 2, 9, False), ("f64", 3, 11, False),
                                                  ("f32", 3, 70, False), ("f64", 2, 8, True), ("f32", 2, 13, True),
                                                  ("f64", 2, 9, "nolayer_x"), ("f32", 2, 6, "nolayer_x")])
def test_adjoint_matches_oracle(dtype, ndim, every, wide):
    """Checkpoint spacings odd and even, so the reverse sweep takes both
    two-step passes and single steps."""
    n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps = _shots(
        ndim=ndim, wide=wide is True, nolayer_x=wide == "nolayer_x")
    print("case adjoint %dD %s ckpt_every=%d wide=%s" % (ndim, dtype, every, wide), flush=True)
    B = len(srcs)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=c2, dtype=tdt, batch=B)
    cells = int(np.prod(N))
    sim.set_state(torch.zeros(sim.shape, dtype=torch.float64))
    sim.inject([b * cells + srcs[b][0] for b in range(B)], torch.from_numpy(wav))
    tr = sim.record([b * cells + r for b in range(B) for r in rec], steps)
    sim.forward_checkpointed(steps, every)
    sim.sync()
    traces = tr.double().cpu().numpy().reshape(B, len(rec), steps)
    resid = traces - obs
    gc2, gw = sim.adjoint(torch.from_numpy(resid.reshape(B * len(rec), steps)))
    sim.sync()
    ogc2, ogw, otr = _oracle_grads(n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps)
    errs = {"traces": _rel(traces, otr), "grad_c2": _rel(gc2.cpu().numpy(), ogc2),
            "grad_w": _rel(gw.double().cpu().numpy(), ogw)}
    print("errors:", {k: "%.2e" % v for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= TOL[dtype], (k, v)
    # a second adjoint call with another residual reuses the checkpoints
    gc2b, _ = sim.adjoint(torch.from_numpy(2.0 * resid.reshape(B * len(rec), steps)))
    sim.sync()
    assert _rel(gc2b.cpu().numpy(), 2.0 * ogc2) <= TOL[dtype]
    sim.close()


def test_autograd_function_matches_oracle():
    from paper_1804_01390_amd.adjoint import ShotProblem, receiver_traces
    n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps = _shots(ndim=2, batch=2, seed=4)
    prob = ShotProblem(n, lo, hi, 1.0, dt, sig, srcs, rec, steps, dtype=torch.float64, ckpt_every=10)
    c2t = torch.tensor(c2, dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(wav, dtype=torch.float64, requires_grad=True)
    tr = receiver_traces(prob, c2t, wt)
    loss = 0.5 * ((tr.cpu() - torch.from_numpy(obs)) ** 2).sum()
    loss.backward()
    ogc2, ogw, otr = _oracle_grads(n, lo, hi, N, sig, c2, dt, srcs, rec, wav, obs, steps)
    assert _rel(tr.detach().cpu().numpy(), otr) <= 1e-12
    assert _rel(c2t.grad.numpy(), ogc2) <= 1e-12
    assert _rel(wt.grad.numpy(), ogw) <= 1e-12


def _pass_case(with_sources):
    """2D 150x130 interior, 3 shots, c^2 field: sources (if any) far enough
    inside the core for passes of up to 8 levels, receivers on a row; no
    sources: a nonzero start instead."""
    rng = np.random.default_rng(21)
    n, lo, hi = [150, 130], [12, 9], [10, 11]
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    sig = [synthetic.sigma_ramp(n[a], lo[a], hi[a], 2.0) for a in range(2)]
    c2 = synthetic.smooth_c2(n, lo, hi, 4, 10.0, 30.0, 0.4, 3, rng)
    dt = 0.5 / np.sqrt(1.4)
    steps, B = 61, 3
    cells = N[0] * N[1]
    srcs = [b * cells + synthetic.flat_index(N, [lo[0] + 30 + 17 * b, lo[1] + 40]) for b in range(B)]
    wav = np.stack([synthetic.ricker(steps, dt, 0.1, 15.0) * (1.0 + 0.3 * b) for b in range(B)])
    rec = [b * cells + synthetic.flat_index(N, [x, lo[1] + 90]) for b in range(B) for x in range(lo[0], lo[0] + n[0], 2)]
    U0 = None if with_sources else synthetic.gaussian_sum(n, lo, hi, 6, 3.0, 8.0, rng)
    resid = rng.normal(scale=1e-2, size=(len(rec), steps))
    return n, lo, hi, sig, c2, dt, steps, B, srcs, wav, rec, U0, resid


def _adjoint_run(case, dtype, variant, tile_rows, every):
    n, lo, hi, sig, c2, dt, steps, B, srcs, wav, rec, U0, resid = case
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=c2, dtype=tdt, batch=B)
    sim.set_variant(variant, tile_rows)
    if U0 is None:
        sim.set_state(torch.zeros(sim.shape, dtype=torch.float64))
        sim.inject(srcs, torch.from_numpy(wav))
    else:
        sim.set_state(torch.stack([torch.from_numpy(U0) * (1.0 + 0.5 * b) for b in range(B)]))
    tr = sim.record(rec, steps)
    sim.forward_checkpointed(steps, every)
    sim.sync()
    traces = tr.cpu().numpy().copy()
    gc2, gw = sim.adjoint(torch.from_numpy(resid))
    sim.sync()
    out = [traces, gc2.cpu().numpy()] + ([gw.cpu().numpy()] if gw is not None else [])
    sim.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("with_sources", [True, False])
@pytest.mark.parametrize("every", [13, 20])
def test_adjoint_recompute_passes_bit_identical(dtype, with_sources, every):
    """The adjoint's recompute as multi-step passes that keep every level
    (with the sources added inside them) gives the single-step history: the
    traces and both gradients equal a one-thread-per-cell run bit for bit."""
    case = _pass_case(with_sources)
    print("case adjoint passes %s sources=%s every=%d" % (dtype, with_sources, every), flush=True)
    ref = _adjoint_run(case, dtype, dp.VARIANT_CELL, 0, every)
    for variant, tile_rows in ((dp.VARIANT_DEEP, 8 << 20), (dp.VARIANT_DEEP, (6 << 20) | (4 << 12) | 16),
                               (dp.VARIANT_DEEP, (5 << 20) | (1 << 12) | 24), (dp.VARIANT_FOURSTEP, 7),
                               (dp.VARIANT_THREESTEP, 8), (dp.VARIANT_TWOSTEP, (3 << 16) | 8)):
        got = _adjoint_run(case, dtype, variant, tile_rows, every)
        for k, (a, b) in enumerate(zip(got, ref)):
            assert np.array_equal(a, b), (variant, hex(tile_rows), k)
