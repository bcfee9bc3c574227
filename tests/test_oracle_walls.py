"""Pins of the oracle's reflecting-wall truncation (the case the paper
analyses with Eq. (IntroReflectedDecayBound)): Dirichlet sine modes, energy
conservation, no interface reflection before the wall echo returns, and an
echo that falls exponentially as the layer thickens."""
import math

import numpy as np
import pytest

import oracle
import synthetic
from oracle import closed_forms as cf


@pytest.mark.parametrize("ndim,dt", [(1, 0.9), (2, 0.5), (3, 0.4)])
def test_dirichlet_sine_modes_exact(ndim, dt):
    N = [21, 17, 13][:ndim]
    m = [3, 2, 4][:ndim]
    k = [math.pi * m[a] / (N[a] + 1) for a in range(ndim)]
    X = np.meshgrid(*[np.arange(n) for n in reversed(N)], indexing="ij")[::-1]
    U0 = np.ones(tuple(reversed(N)))
    for a in range(ndim):
        U0 = U0 * np.sin(k[a] * (X[a] + 1))
    g = oracle.Grid(N, 1.0, dt, [np.zeros(n) for n in N], walls=[True] * ndim)
    theta = cf.leapfrog_theta(k, 1.0, dt)
    fin, _ = oracle.run(g, oracle.start(g, U0), 250)
    assert np.max(np.abs(fin.U - math.cos(250 * theta) * U0)) < 5e-13


def test_energy_conserved_with_walls():
    rng = np.random.default_rng(9)
    n = [33, 29]
    U0 = synthetic.gaussian_sum(n, [0, 0], [0, 0], 10, 2.0, 4.0, rng)
    g = oracle.Grid(n, 1.0, 0.5, [np.zeros(33), np.zeros(29)], walls=[True, True])
    s = oracle.start(g, U0)
    es = []
    for _ in range(4):
        s2, _ = oracle.run(g, s, 150)
        one, _ = oracle.run(g, s2, 1)
        es.append(cf.leapfrog_energy(one.U, s2.U, 1.0, 0.5, walls=True))
        s = s2
    es = np.array(es)
    assert np.max(np.abs(es - es[0])) / es[0] < 1e-13


def _wall_vs_free(n, m, steps, sig, width):
    N = n + 2 * m
    g = oracle.Grid([N, N], 1.0, 0.5, [sig, sig.copy()], walls=[True, True])
    fin, _ = oracle.run(g, oracle.start(g, synthetic.gaussian_bump([n, n], [m, m], [m, m], width)), steps)
    Nr = n + 2 * (steps + 4)
    off = (Nr - n) // 2
    gr = oracle.Grid([Nr, Nr], 1.0, 0.5, [None, None])
    sr = oracle.start(gr, synthetic.gaussian_bump([n, n], [off, off], [Nr - n - off] * 2, width))
    Ur, _ = oracle.wave_run(gr, sr.U, sr.Uprev, steps)
    return np.max(np.abs(fin.U[m:m + n, m:m + n] - Ur[off:off + n, off:off + n])) / np.max(np.abs(sr.U))


def test_wall_truncated_layer_reflects_nothing_at_the_interface():
    # 40-cell layers, 70 steps: the echo from the wall cannot be back yet
    n, m = 80, 40
    err = _wall_vs_free(n, m, 70, synthetic.sigma_const(n, m, m, 2.0), 4.0)
    assert err < 1e-13


def test_wall_echo_decays_exponentially_with_thickness():
    n, steps = 64, 220
    errs = [_wall_vs_free(n, m, steps, synthetic.sigma_const(n, m, m, 1.0), 3.0) for m in (3, 6, 9, 12)]
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < 2e-2 * a or b < 1e-15
    # a bare wall (no layer) reflects at O(1)
    assert _wall_vs_free(n, 1, steps, np.zeros(n + 2), 3.0) > 1e-2
