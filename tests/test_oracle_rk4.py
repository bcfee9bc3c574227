"""Pins of the oracle's RK4 integrator (the paper's own time stepping,
Sec. 1.1.3): the semi-discrete layer modes of Thm. 1 are eigenvectors of one
RK4 step, periodic Fourier modes evolve by Re(P(-i omega dt)^n), and the
truncated run matches the RK4 free-space run (Figs. 2/3)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synthetic
from oracle import closed_forms as cf


def _part(mode, part):
    return oracle.RKState(part(mode["U"]).copy(), part(mode["V"]).copy(),
                          [part(p).copy() for p in mode["Phi"]], [part(p).copy() for p in mode["Psi"]])


@pytest.mark.parametrize("k", [(0.6, 0.3), (2.2, 1.4), (0.4 + 0.15j, 0.8)])
def test_rk4_layer_mode_is_exact_eigenvector(k):
    rng = np.random.default_rng(12)
    N, b, h, dt = [26, 22], [11, 10], 1.0, 0.3
    sig = []
    for a in range(2):
        s = np.zeros(N[a])
        s[b[a]:] = rng.uniform(0.0, 2.0, size=N[a] - b[a])
        sig.append(s)
    mode = cf.semidiscrete_layer_mode(N, b, sig, k, h)
    fac = cf.rk4_factor(-1j * mode["omega"] * dt)
    g = oracle.Grid(N, h, dt, sig)
    # one RK4 step reads up to 4 cells away (four nested stencil applications)
    inner = (slice(4, -4), slice(4, -4))
    scale = max(1.0, np.max(np.abs(mode["U"])))
    for part in (np.real, np.imag):
        s1 = oracle.rk4_run(g, _part(mode, part), 1)
        assert np.max(np.abs(s1.U - part(fac * mode["U"]))[inner]) <= 1e-13 * scale
        assert np.max(np.abs(s1.V - part(fac * mode["V"]))[inner]) <= 1e-13 * scale
        for a in range(2):
            assert np.max(np.abs(s1.Phi[a] - part(fac * mode["Phi"][a]))[inner]) <= 1e-13 * scale
            assert np.max(np.abs(s1.Psi[a] - part(fac * mode["Psi"][a]))[inner]) <= 1e-13 * scale


def test_rk4_fourier_mode():
    N = [24, 20]
    k = [2 * math.pi * 3 / 24, 2 * math.pi * 2 / 20]
    X = np.meshgrid(np.arange(20), np.arange(24), indexing="ij")[::-1]
    U0 = np.cos(k[0] * X[0] + k[1] * X[1])
    g = oracle.Grid(N, 1.0, 0.4, [np.zeros(24), np.zeros(20)])
    w = 2.0 * math.sqrt(math.sin(k[0] / 2) ** 2 + math.sin(k[1] / 2) ** 2)
    P = cf.rk4_factor(-1j * w * 0.4)
    s = oracle.rk4_run(g, oracle.rk4_start(g, U0), 100)
    assert np.max(np.abs(s.U - np.real(P ** 100) * U0)) < 1e-12


def test_rk4_reflectionless_fig2_setup():
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_setups.json")) as f:
        cfg = json.load(f)["fig2"]
    n, m, steps, dt = cfg["interior_cells"], cfg["layer_cells_per_side"], cfg["steps"] // 2, 0.5
    sig = synthetic.sigma_const(n, m, m, cfg["sigma_h"])
    N = n + 2 * m
    g = oracle.Grid([N, N], 1.0, dt, [sig, sig.copy()])
    U0 = synthetic.gaussian_bump([n, n], [m, m], [m, m], cfg["bump_width"], amp=cfg["bump_peak"])
    fin = oracle.rk4_run(g, oracle.rk4_start(g, U0), steps)
    Nr = n + 2 * (4 * steps + 4)
    off = (Nr - n) // 2
    gr = oracle.Grid([Nr, Nr], 1.0, dt, [None, None])
    U0r = synthetic.gaussian_bump([n, n], [off, off], [Nr - n - off] * 2, cfg["bump_width"], amp=cfg["bump_peak"])
    ref = oracle.rk4_run(gr, oracle.rk4_start(gr, U0r), steps)
    a = fin.U[m:m + n, m:m + n]
    r = ref.U[off:off + n, off:off + n]
    assert np.max(np.abs(a - r)) / np.max(np.abs(r)) < 1e-13
