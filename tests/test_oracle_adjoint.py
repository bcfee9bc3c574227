"""Pins of the oracle's discrete adjoint against the (pinned) forward oracle:
the map from wavelets to receiver traces is linear, so its transpose must
satisfy the dot-product identity to rounding; the c^2 gradient must match
central differences of the misfit."""
import numpy as np
import pytest

import oracle
import synthetic


def _problem(seed=0, steps=60, c2_field=True):
    rng = np.random.default_rng(seed)
    n, lo, hi = [30, 26], [6, 5], [5, 7]
    N = [lo[a] + n[a] + hi[a] for a in range(2)]
    sig = [synthetic.sigma_random(n[a], lo[a], hi[a], 2.0, rng) for a in range(2)]
    c2 = synthetic.smooth_c2(n, lo, hi, 4, 3.0, 6.0, 0.4, 3, rng) if c2_field else None
    g = oracle.Grid(N, 1.0, 0.45, sig, c2=c2)
    src = [synthetic.flat_index(N, [lo[0] + 5, lo[1] + 4]), synthetic.flat_index(N, [lo[0] + 20, lo[1] + 9])]
    rec = [synthetic.flat_index(N, [lo[0] + x, lo[1] + 18]) for x in range(2, 28, 3)]
    rec.append(synthetic.flat_index(N, [2, 3]))       # a receiver inside the layer
    rec.append(src[0])                                 # and one on a source
    wav = np.vstack([synthetic.ricker(steps, 0.45, 0.12, 8.0), synthetic.ricker(steps, 0.45, 0.09, 11.0)])
    U0 = synthetic.gaussian_bump(n, lo, hi, 2.5, amp=0.3)
    return g, U0, src, rec, wav, steps


def _traces(g, U0, src, rec, wav, steps):
    _, tr = oracle.run(g, oracle.start(g, U0), steps, sources=src, wavelets=wav, receivers=rec, nt=steps)
    return tr


def test_adjoint_dot_product_identity_for_wavelets():
    g, U0, src, rec, wav, steps = _problem()
    rng = np.random.default_rng(1)
    dw = rng.normal(size=wav.shape)
    y = rng.normal(size=(len(rec), steps))
    # F dw with zero initial field: the linear part of the trace map
    Fdw = _traces(g, np.zeros_like(U0), src, rec, dw, steps)
    _, FTy = oracle.adjoint(g, np.zeros_like(U0), steps, src, dw, rec, y)
    lhs = float(np.sum(Fdw * y))
    rhs = float(np.sum(dw * FTy))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


def test_adjoint_c2_gradient_matches_central_differences():
    g, U0, src, rec, wav, steps = _problem(seed=3)
    rng = np.random.default_rng(2)
    obs = _traces(g, U0, src, rec, wav, steps) * 0.9 + 1e-3 * rng.normal(size=(len(rec), steps))

    def J(c2):
        gg = oracle.Grid(g.N, g.h, g.dt, g.sigma, c2=c2)
        d = _traces(gg, U0, src, rec, wav, steps)
        return 0.5 * float(np.sum((d - obs) ** 2))

    d0 = _traces(g, U0, src, rec, wav, steps)
    gc2, gw = oracle.adjoint(g, U0, steps, src, wav, rec, d0 - obs)
    # a smooth perturbation supported away from the layer
    n, lo = [30, 26], [6, 5]
    dc = synthetic.gaussian_bump(n, lo, [5, 7], 4.0, center=[14.0, 12.0])
    eps = 1e-4
    fd = (J(g.c2 + eps * dc) - J(g.c2 - eps * dc)) / (2 * eps)
    ad = float(np.sum(gc2 * dc))
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    # single-cell perturbations, including one next to the layer
    for cell in [(20, 20), (12, 7), (30, 11)]:
        e = np.zeros_like(g.c2)
        e[cell] = 1.0
        fd1 = (J(g.c2 + eps * e) - J(g.c2 - eps * e)) / (2 * eps)
        assert abs(fd1 - gc2[cell]) <= 1e-6 * max(abs(fd1), 1e-12) + 1e-14
    # wavelet gradient against differences too (quadratic in w: exact)
    def Jw(w):
        d = _traces(g, U0, src, rec, w, steps)
        return 0.5 * float(np.sum((d - obs) ** 2))
    for s, k in [(0, 10), (1, 33), (0, steps - 1)]:
        e = np.zeros_like(wav)
        e[s, k] = 1.0
        fdw = (Jw(wav + 1e-3 * e) - Jw(wav - 1e-3 * e)) / 2e-3
        assert abs(fdw - gw[s, k]) <= 1e-8 * max(abs(fdw), 1e-10)
