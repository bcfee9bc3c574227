"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the
oracle: damping profiles, initial fields, wave-speed fields, source wavelets
and receiver sets.  This module holds none of the scheme's arithmetic; it only
draws and lays out input arrays (host FP64 numpy).

Conventions: per-axis extents are given in the paper's axis order (x, y, z);
field arrays have numpy shape reversed (z, y, x) so x is the fastest axis.
An axis with ``n`` interior cells and layer widths ``lo`` (low side) and
``hi`` (high side) has ``N = lo + n + hi`` cells; the interior is
``[lo, lo + n)`` and, with periodic wrap, the layer is the single band
``[lo + n, N) U [0, lo)`` (the physical box "surrounded" by one layer, as in
the runs of Figs. 2 and 3 of the paper).  A damping value sigma(i) belongs to
the edge [i, i+1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


# ----------------------------------------------------------------------------
# damping profiles (one array of length N per axis)
# ----------------------------------------------------------------------------

def sigma_ramp(n: int, lo: int, hi: int, smax: float, power: float = 2.0) -> np.ndarray:
    """Profile rising from 0 at each interface to ``smax`` at the array ends:
    the edge at distance d (d = 0 touches the interface) into a side of width
    m gets smax * ((d + 1/2)/m)^power."""
    N = lo + n + hi
    s = np.zeros(N)
    for d in range(hi):
        s[lo + n + d] = smax * ((d + 0.5) / hi) ** power
    for d in range(lo):
        s[lo - 1 - d] = smax * ((d + 0.5) / lo) ** power
    return s


def sigma_const(n: int, lo: int, hi: int, value: float) -> np.ndarray:
    """Constant damping on every layer edge (Fig. 2 setup)."""
    N = lo + n + hi
    s = np.zeros(N)
    s[lo + n:] = value
    s[:lo] = value
    return s


def sigma_random(n: int, lo: int, hi: int, smax: float, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. Uniform[0, smax] damping on every layer edge (Fig. 3 setup)."""
    N = lo + n + hi
    s = np.zeros(N)
    s[lo + n:] = rng.uniform(0.0, smax, size=hi)
    s[:lo] = rng.uniform(0.0, smax, size=lo)
    return s


# ----------------------------------------------------------------------------
# initial fields
# ----------------------------------------------------------------------------

def _coords(N: Sequence[int]):
    """Index grids (x, y, z order) for a box of extents N."""
    axes = [np.arange(n, dtype=np.float64) for n in N]
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))


def embed(inner: np.ndarray, n, lo, hi) -> np.ndarray:
    """Place an interior-box array (numpy shape reversed(n)) into a zero field
    of extents lo + n + hi.  Generators draw on the interior box only, so the
    same seed gives bit-identical interior data whatever the layer widths."""
    d = len(n)
    N = [lo[a] + n[a] + hi[a] for a in range(d)]
    out = np.zeros(tuple(reversed(N)))
    sl = tuple(slice(lo[a], lo[a] + n[a]) for a in reversed(range(d)))
    out[sl] = inner
    return out


def interior_mask(n: Sequence[int], lo: Sequence[int], hi: Sequence[int]) -> np.ndarray:
    return embed(np.ones(tuple(reversed(list(n)))), n, lo, hi) > 0


def gaussian_bump(n, lo, hi, width: float, center=None, amp: float = 1.0) -> np.ndarray:
    """amp * exp(-|x - x_c|^2 / (2 width^2)) on the interior, zero outside.
    ``center`` is in interior coordinates (default (n - 1)/2 on every axis)."""
    d = len(n)
    if center is None:
        center = [(n[a] - 1) / 2.0 for a in range(d)]
    X = _coords(n)
    r2 = sum((X[a] - center[a]) ** 2 for a in range(d))
    return embed(amp * np.exp(-r2 / (2.0 * width * width)), n, lo, hi)


def gaussian_sum(n, lo, hi, count: int, wmin: float, wmax: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Sum of ``count`` Gaussians on the interior: widths ~ U(wmin, wmax),
    amplitudes ~ N(0,1), centres uniform over the interior box; drawn in the
    order (widths, amplitudes, x centres, y centres, z centres).  Zero outside
    the interior."""
    d = len(n)
    w = rng.uniform(wmin, wmax, size=count)
    amp = rng.normal(0.0, 1.0, size=count)
    ctr = [rng.uniform(0.0, n[a], size=count) for a in range(d)]
    X = _coords(n)
    U = np.zeros(tuple(reversed(list(n))))
    for q in range(count):
        # evaluate inside a +-9 width box (the Gaussian is below 1e-17 beyond)
        sl = []
        for a in reversed(range(d)):
            r = 9.0 * w[q]
            a0 = max(0, int(math.floor(ctr[a][q] - r)))
            a1 = min(n[a], int(math.ceil(ctr[a][q] + r)) + 1)
            sl.append(slice(a0, a1))
        sl = tuple(sl)
        r2 = sum((X[a][sl] - ctr[a][q]) ** 2 for a in range(d))
        U[sl] += amp[q] * np.exp(-r2 / (2.0 * w[q] ** 2))
    return embed(U, n, lo, hi)


def white_noise_disk(n, lo, hi, radius: float, variance: float,
                     rng: np.random.Generator) -> np.ndarray:
    """i.i.d. N(0, variance) values on the cells of a disk (ball) of the given
    radius about the interior centre, zero elsewhere (Fig. 3 setup).  The
    draws cover the interior box in x-fastest order."""
    d = len(n)
    X = _coords(n)
    ctr = [(n[a] - 1) / 2.0 for a in range(d)]
    r2 = sum((X[a] - ctr[a]) ** 2 for a in range(d))
    U = rng.normal(0.0, math.sqrt(variance), size=tuple(reversed(list(n))))
    U[r2 > radius * radius] = 0.0
    return embed(U, n, lo, hi)


def smooth_c2(n, lo, hi, count: int, wmin: float, wmax: float, contrast: float,
              margin: int, rng: np.random.Generator) -> np.ndarray:
    """c^2 = 1 + contrast * g, g a sum of ``count`` Gaussians (widths U(wmin,
    wmax), amplitudes N(0,1), centres uniform over the interior) scaled to
    max|g| = 1 and forced to 0 on the layer and within ``margin`` cells of it."""
    d = len(n)
    g = gaussian_sum(n, [0] * d, [0] * d, count, wmin, wmax, rng)
    m = np.max(np.abs(g))
    if m > 0:
        g = g / m
    keep = embed(np.ones(tuple(reversed([n[a] - 2 * margin for a in range(d)]))),
                 [n[a] - 2 * margin for a in range(d)], [margin] * d, [margin] * d) > 0
    g[~keep] = 0.0
    return 1.0 + contrast * embed(g, n, lo, hi)


# ----------------------------------------------------------------------------
# sources
# ----------------------------------------------------------------------------

def ricker(nt: int, dt: float, f: float, t0: float) -> np.ndarray:
    """Ricker wavelet samples w(t_n), t_n = n dt:
    (1 - 2 pi^2 f^2 (t - t0)^2) exp(-pi^2 f^2 (t - t0)^2)."""
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def flat_index(N: Sequence[int], idx: Sequence[int]) -> int:
    """Flat cell index of (x, y, z) with x fastest."""
    f = 0
    stride = 1
    for a in range(len(N)):
        f += int(idx[a]) * stride
        stride *= int(N[a])
    return f


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    """One synthetic problem.  ``n``, ``lo``, ``hi`` per axis (x, y, z order)."""
    name: str
    n: List[int]
    lo: List[int]
    hi: List[int]
    h: float
    dt: float
    steps: int
    sigma: List[np.ndarray]
    U0: Optional[np.ndarray]
    c2: Optional[np.ndarray] = None
    sources: List[int] = field(default_factory=list)
    wavelets: Optional[np.ndarray] = None        # [ns][nt]
    receivers: List[int] = field(default_factory=list)
    plane: Optional[tuple] = None                # (axis, index) of a recorded plane

    @property
    def N(self) -> List[int]:
        return [self.lo[a] + self.n[a] + self.hi[a] for a in range(len(self.n))]

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def cells(self) -> int:
        return int(np.prod(self.N))


def bump2d(n=128, m=16, steps: int = 500, smax: float = 2.0,
           width: float = 4.0, h: float = 1.0, courant: float = 0.5) -> Workload:
    """2D, n x n interior + m-cell layer on each side, h = 1, c = 1,
    dt = courant * h, quadratic ramp to smax, centred Gaussian bump (zero
    velocity).  ``n`` may be a pair (nx, ny) for a rectangular interior.
    Defaults: the 128^2 + 16-cell, 500-step parity case."""
    nx, ny = (n, n) if np.isscalar(n) else (int(n[0]), int(n[1]))
    sx = sigma_ramp(nx, m, m, smax)
    sy = sigma_ramp(ny, m, m, smax)
    U0 = gaussian_bump([nx, ny], [m, m], [m, m], width)
    name = "bump2d_%d_m%d" % (nx, m) if nx == ny else "bump2d_%dx%d_m%d" % (nx, ny, m)
    return Workload(name, [nx, ny], [m, m], [m, m], h, courant * h, steps, [sx, sy], U0)


def bumps2d(n: int = 4096, m: int = 32, steps: int = 2000, seed: int = 0,
            count: int = 64, courant: float = 0.5, h: float = 1.0, margin: int = 0) -> Workload:
    """2D, n x n interior + m-cell layer per side, c = 1, dt = courant * h,
    quadratic ramp to 2/h, U0 = sum of ``count`` Gaussians (widths U(2,8) h,
    amplitudes N(0,1), uniform centres) from ``seed``.  Defaults: the
    4096^2 + 32-cell, 2000-step throughput case.  ``margin`` > 0 also zeroes
    U0 on the ``margin`` interior cells next to every layer interface (data
    that starts in the physical domain, away from the layer: the setting of
    the free-space reflection measurement)."""
    rng = np.random.default_rng(seed)
    sig = sigma_ramp(n, m, m, 2.0 / h)
    U0 = gaussian_sum([n, n], [m, m], [m, m], count, 2.0, 8.0, rng)
    if margin > 0:
        keep = np.zeros_like(U0, dtype=bool)
        keep[m + margin:m + n - margin, m + margin:m + n - margin] = True
        U0[~keep] = 0.0
    return Workload("bumps2d_%d_m%d" % (n, m), [n, n], [m, m], [m, m], h, courant * h,
                    steps, [sig, sig.copy()], U0)


def ricker3d(n: int = 512, m: int = 24, steps: int = 1000, courant: float = 0.4,
             h: float = 1.0, ppw: float = 15.0, record_plane: bool = True) -> Workload:
    """3D, n^3 interior + m-cell layer on all six faces, c = 1,
    dt = courant * h, quadratic ramp to 2/h, zero initial field, one Ricker
    point source at the interior centre cell (n/2, n/2, n/2) with peak
    frequency f = 1/(ppw h) and delay 1.5/f, recording the z plane through
    the source.  Defaults: the 512^3 + 24-cell, 1000-step case."""
    sig = sigma_ramp(n, m, m, 2.0 / h)
    N = [m + n + m] * 3
    dt = courant * h
    f = 1.0 / (ppw * h)
    src = flat_index(N, [m + n // 2] * 3)
    wav = ricker(steps, dt, f, 1.5 / f)[None, :]
    plane = (2, m + n // 2) if record_plane else None
    return Workload("ricker3d_%d_m%d" % (n, m), [n] * 3, [m] * 3, [m] * 3, h, dt, steps,
                    [sig, sig.copy(), sig.copy()], None, sources=[src], wavelets=wav,
                    plane=plane)


def batch2d(count: int = 256, seed: int = 0, steps: int = 1500, smin: int = 256,
            smax_side: int = 1536, mmin: int = 16, mmax: int = 32,
            courant: float = 0.5) -> List[Workload]:
    """``count`` independent 2D problems: each of the two interior sides
    round(exp(U(ln smin, ln smax))) drawn independently (x sides first, then
    y sides), layer width uniform in {mmin..mmax}, quadratic ramp to 2/h, one
    centred Gaussian (width 4) each."""
    rng = np.random.default_rng(seed)
    sx = np.round(np.exp(rng.uniform(math.log(smin), math.log(smax_side), size=count))).astype(int)
    sy = np.round(np.exp(rng.uniform(math.log(smin), math.log(smax_side), size=count))).astype(int)
    ms = rng.integers(mmin, mmax + 1, size=count)
    out = []
    for b in range(count):
        w = bump2d((int(sx[b]), int(sy[b])), int(ms[b]), steps, 2.0, 4.0, 1.0, courant)
        w.name = "batch%d_%dx%d_m%d" % (b, sx[b], sy[b], ms[b])
        out.append(w)
    return out


@dataclass
class ShotWorkload:
    """A batch of shots on one 2D grid for the adjoint: shared c^2 (model and
    'true'), one Ricker source per shot, receivers shared by all shots."""
    n: List[int]
    lo: List[int]
    hi: List[int]
    h: float
    dt: float
    steps: int
    sigma: List[np.ndarray]
    c2_model: np.ndarray
    c2_true: np.ndarray
    sources: List[List[int]]        # per shot, flat cells within one member
    receivers: List[int]            # flat cells within one member
    wavelets: np.ndarray            # [shots][steps]

    @property
    def N(self) -> List[int]:
        return [self.lo[a] + self.n[a] + self.hi[a] for a in range(len(self.n))]

    @property
    def cells(self) -> int:
        return int(np.prod(self.N))


def shots2d(n: int = 1024, m: int = 32, shots: int = 32, steps: int = 3000, seed: int = 0,
            src_row: int = 16, rec_row: int = 24, spacing: int = 32, ppw: float = 15.0,
            count: int = 32, wmin: float = 20.0, wmax: float = 80.0, margin: int = 8) -> ShotWorkload:
    """2D, n^2 interior + m-cell layer, c^2 = 1 + 0.5 g (g: ``count`` seeded
    Gaussians of widths U(wmin, wmax), scaled to max|g| = 1, held at 0 within
    ``margin`` cells of the layer); a second seed gives the 'true' c^2.
    ``shots`` Ricker sources on interior row ``src_row`` at x = 16 + spacing*s
    (f = 1/(ppw h), delay 1.5/f), receivers on every interior cell of row
    ``rec_row``, dt = 0.5 h / c_max.  Defaults: the 1024^2 + 32-cell,
    32-shot, 3000-step adjoint case."""
    rng = np.random.default_rng(seed)
    c2m = smooth_c2([n, n], [m, m], [m, m], count, wmin, wmax, 0.5, margin, rng)
    c2t = smooth_c2([n, n], [m, m], [m, m], count, wmin, wmax, 0.5, margin,
                    np.random.default_rng(seed + 1))
    h = 1.0
    cmax = math.sqrt(max(float(np.max(c2m)), float(np.max(c2t))))
    dt = 0.5 * h / cmax
    sig = sigma_ramp(n, m, m, 2.0 / h)
    N = [m + n + m] * 2
    srcs = [[flat_index(N, [m + 16 + spacing * s, m + src_row])] for s in range(shots)]
    rec = [flat_index(N, [m + x, m + rec_row]) for x in range(n)]
    f = 1.0 / (ppw * h)
    wav = np.vstack([ricker(steps, dt, f, 1.5 / f) for _ in range(shots)])
    return ShotWorkload([n, n], [m, m], [m, m], h, dt, steps, [sig, sig.copy()], c2m, c2t, srcs, rec, wav)
