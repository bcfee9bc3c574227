"""The 2D adjoint frame at the 4 GiB boundary: the frame reaches a batch's
arrays through one buffer descriptor per array while every array (all shots
together) stays below 4 GiB, and through per-shot scalar bases past it.  A
34-shot FP64 run on a 4032^2 grid (4.4 GB per field array, the per-shot
form) must equal two 17-shot runs of the same shots (2.2 GB each, the
descriptor form): traces and wavelet gradients bit for bit (every shot's
forward and adjoint fields are formed alone), the c^2 gradient, a sum over
shots whose grouping differs, to FP64 rounding."""
import numpy as np
import pytest

import synthetic

torch = pytest.importorskip("torch")
dp = pytest.importorskip("paper_1804_01390_amd")

pytestmark = pytest.mark.gpu


def _run(n, lo, hi, sig, c2, dt, steps, every, shots, recs, wav, resid):
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    cells = N[0] * N[1]
    B = len(shots)
    sim = dp.Simulation(n, lo, hi, 1.0, dt, sig, c2=c2, dtype=torch.float64, batch=B)
    sim.set_state(torch.zeros(sim.shape, dtype=torch.float64, device="cuda"))
    sim.inject([b * cells + shots[b] for b in range(B)], torch.from_numpy(wav))
    tr = sim.record([b * cells + r for b in range(B) for r in recs[b]], steps)
    sim.forward_checkpointed(steps, every)
    sim.sync()
    traces = tr.cpu().numpy().copy()
    gc2, gw = sim.adjoint(torch.from_numpy(resid))
    sim.sync()
    out = traces, gc2.cpu().numpy(), gw.cpu().numpy()
    sim.close()
    del tr, gc2, gw, sim
    torch.cuda.empty_cache()
    return out


def test_adjoint_frame_past_4gib_equals_two_halves():
    n, lo, hi = [4000, 4000], [16, 16], [16, 16]
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    B, steps, every, dt = 34, 8, 3, 0.5
    assert B * N[0] * N[1] * 8 >= 1 << 32 > (B // 2) * N[0] * N[1] * 8
    rng = np.random.default_rng(5)
    sig = [synthetic.sigma_ramp(n[a], lo[a], hi[a], 2.0) for a in range(2)]
    # a c^2 field (the c^2 gradient is formed for a field only)
    c2 = synthetic.smooth_c2(n, lo, hi, 6, 300.0, 900.0, 0.4, 2, rng)
    # sources in the core and inside the layer (cells the frame steps), the
    # receivers of each shot a few cells around its source (the wave reaches
    # them within the run), some of them in the layer
    pos = [(lo[0] + 2 + 117 * b, lo[1] + 3 + 97 * b) for b in range(B - 2)] + [(3, 5), (N[0] - 2, 40)]
    shots = [synthetic.flat_index(N, p) for p in pos]
    offs = [(3, 0), (0, 4), (-5, 2), (2, -6), (-1, -3)]
    recs = [[synthetic.flat_index(N, [(x + dx) % N[0], (y + dy) % N[1]]) for dx, dy in offs] for x, y in pos]
    wav = np.stack([synthetic.ricker(steps, dt, 0.1, 1.0 + 0.1 * b) for b in range(B)])
    nr = len(offs)
    resid = rng.normal(size=(B * nr, steps))
    print("case adjoint 4032^2 FP64, %d shots vs two halves, %d steps" % (B, steps), flush=True)
    full = _run(n, lo, hi, sig, c2, dt, steps, every, shots, recs, wav, resid)
    h = B // 2
    a = _run(n, lo, hi, sig, c2, dt, steps, every, shots[:h], recs[:h], wav[:h], resid[:h * nr])
    b = _run(n, lo, hi, sig, c2, dt, steps, every, shots[h:], recs[h:], wav[h:], resid[h * nr:])
    assert np.array_equal(full[0], np.concatenate([a[0], b[0]]))
    assert np.array_equal(full[2], np.concatenate([a[2], b[2]]))
    g = a[1] + b[1]
    assert np.max(np.abs(g)) > 0
    err = float(np.max(np.abs(full[1] - g)) / np.max(np.abs(g)))
    print("grad_c2 rel err %.2e" % err, flush=True)
    assert err <= 1e-13
