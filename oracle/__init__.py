"""Plain FP64 CPU oracle for the reflectionless discrete PML (Chern,
"A Reflectionless Discrete Perfectly Matched Layer", arXiv 1804.01390).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

The arithmetic lives in ``dpml_oracle.c`` (compiled with gcc, ``-O2
-ffp-contract=off``, OpenMP over cells).  This module only marshals numpy
arrays in and out.  Arrays are numpy FP64 with shape ``(N2, N1, N0)`` for 3D,
``(N1, N0)`` for 2D and ``(N0,)`` for 1D: axis 0 of the paper's grid (x) is
the LAST (fastest) numpy axis.

Parity status of each function (see the pins in ``tests/test_oracle_pins.py``):
  start                  -- pinned: both branches.  Zero velocity: exact
                            Fourier modes at rest (U^{-1} = cos(theta) U^0).
                            Given velocity V^0: the exact leapfrog sine/cosine
                            mode a cos(n theta) + (dt v / sin theta) sin(n theta)
                            (Sec. 1.1.1, Eq. DiscreteDispersion)
  step, run              -- pinned (exact Fourier modes, Sec. 1.1.1 / Eq.
                            DiscreteDispersion; exact layer modes of Thm. 1;
                            energy conservation; reflection against free space,
                            Figs. 2/3; 1-D light-cone Green's function)
  wave_run               -- pinned (exact Fourier modes)
  rk4_run                -- pinned (exact one-step layer eigenmodes of the
                            semi-discrete system, Fourier modes, reflection
                            against the RK4 free-space run)
  adjoint                -- pinned (dot-product identity for the wavelet map,
                            which is linear; central differences for c^2)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpml_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/_liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("N", ctypes.c_int64 * 3),
        ("h", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("c2", ctypes.POINTER(ctypes.c_double)),
        ("sigma", ctypes.POINTER(ctypes.c_double) * 3),
        ("wall", ctypes.c_int32 * 3),
        ("pad2_", ctypes.c_int32),
    ]


_DP = ctypes.POINTER(ctypes.c_double)
_DP3 = _DP * 3
_I64P = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        gp = ctypes.POINTER(_Grid)
        lib.orc_start.argtypes = [gp, _DP, _DP, _DP]
        lib.orc_start.restype = None
        lib.orc_step.argtypes = [gp, _DP, _DP, _DP3, _DP3, _DP, _DP3, _DP3]
        lib.orc_step.restype = None
        lib.orc_run.argtypes = [gp, _DP, _DP, _DP3, _DP3, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int64, _I64P, _DP,
                                ctypes.c_int64, _I64P, _DP, ctypes.c_int64]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_wave_run.argtypes = [gp, _DP, _DP, ctypes.c_int64]
        lib.orc_wave_run.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [gp, _DP, ctypes.c_int64, ctypes.c_int64, _I64P, _DP,
                                    ctypes.c_int64, _I64P, _DP, _DP, _DP]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_rk4_run.argtypes = [gp, _DP, _DP, _DP3, _DP3, ctypes.c_int64]
        lib.orc_rk4_run.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return _DP()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


@dataclass
class Grid:
    """Problem description.  ``N`` is given in the paper's axis order
    (x, y, z); ``sigma[a]`` has ``N[a]`` entries (sigma_a(i) lives on the edge
    [i, i+1]); ``c2`` is None (unit speed) or an array of the field shape."""
    N: Sequence[int]
    h: float
    dt: float
    sigma: Sequence[Optional[np.ndarray]] = field(default_factory=list)
    c2: Optional[np.ndarray] = None
    walls: Sequence[bool] = ()     # per axis: True = reflecting walls, else periodic

    @property
    def ndim(self) -> int:
        return len(self.N)

    @property
    def shape(self):
        return tuple(int(n) for n in reversed(list(self.N)))

    def _struct(self):
        g = _Grid()
        g.ndim = self.ndim
        ext = [int(n) for n in self.N] + [1] * (3 - self.ndim)
        for a in range(3):
            g.N[a] = ext[a]
        g.h = float(self.h)
        g.dt = float(self.dt)
        for a in range(3):
            g.wall[a] = 1 if (a < len(self.walls) and self.walls[a]) else 0
        keep = []
        if self.c2 is not None:
            c2 = np.ascontiguousarray(self.c2, dtype=np.float64)
            assert c2.shape == self.shape
            keep.append(c2)
            g.c2 = _dp(c2)
        for a in range(3):
            s = self.sigma[a] if a < len(self.sigma) else None
            if s is not None and a < self.ndim:
                s = np.ascontiguousarray(s, dtype=np.float64)
                assert s.shape == (ext[a],)
                keep.append(s)
                g.sigma[a] = _dp(s)
            else:
                g.sigma[a] = _DP()
        return g, keep


@dataclass
class State:
    """Time level n of the scheme: U^n, U^{n-1} and the auxiliaries Phi_a^n,
    Psi_a^n (full-grid arrays, one per axis)."""
    U: np.ndarray
    Uprev: np.ndarray
    Phi: list
    Psi: list
    n: int = 0

    def copy(self) -> "State":
        return State(self.U.copy(), self.Uprev.copy(), [p.copy() for p in self.Phi],
                     [p.copy() for p in self.Psi], self.n)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _aux3(arrs):
    out = _DP3()
    for a in range(3):
        out[a] = _dp(arrs[a]) if a < len(arrs) else _DP()
    return out


def start(g: Grid, U0, V0=None) -> State:
    """Zero-auxiliary start: U^{-1} = U^0 - dt V^0 + dt^2/2 A(U^0)."""
    lib = _load()
    U0 = _f64(U0).copy()
    assert U0.shape == g.shape
    Um1 = np.empty_like(U0)
    V = None if V0 is None else _f64(V0)
    gs, keep = g._struct()
    lib.orc_start(ctypes.byref(gs), _dp(U0), _dp(V), _dp(Um1))
    zeros = [np.zeros_like(U0) for _ in range(g.ndim)]
    return State(U0, Um1, zeros, [np.zeros_like(U0) for _ in range(g.ndim)], 0)


def step(g: Grid, s: State) -> State:
    """One step of the scheme (no sources); returns a new state."""
    lib = _load()
    gs, keep = g._struct()
    Un = np.empty_like(s.U)
    PhiN = [np.empty_like(s.U) for _ in range(g.ndim)]
    PsiN = [np.empty_like(s.U) for _ in range(g.ndim)]
    Phi = [_f64(p) for p in s.Phi]
    Psi = [_f64(p) for p in s.Psi]
    lib.orc_step(ctypes.byref(gs), _dp(_f64(s.U)), _dp(_f64(s.Uprev)), _aux3(Phi), _aux3(Psi),
                 _dp(Un), _aux3(PhiN), _aux3(PsiN))
    return State(Un, s.U.copy(), PhiN, PsiN, s.n + 1)


def run(g: Grid, s: State, nsteps: int, sources=None, wavelets=None,
        receivers=None, nt: Optional[int] = None):
    """Run ``nsteps`` steps from state ``s`` (not modified).  ``sources`` and
    ``receivers`` are flat cell indices (x fastest); ``wavelets`` is
    ``[ns][nt]``.  Returns ``(state, traces)`` with ``traces`` ``[nr][nt]``
    (column n holds U^{n+1} at the receiver after step n)."""
    lib = _load()
    gs, keep = g._struct()
    out = s.copy()
    out.U = _f64(out.U).copy()
    out.Uprev = _f64(out.Uprev).copy()
    out.Phi = [_f64(p).copy() for p in out.Phi]
    out.Psi = [_f64(p).copy() for p in out.Psi]
    src = np.ascontiguousarray(sources if sources is not None else [], dtype=np.int64)
    rec = np.ascontiguousarray(receivers if receivers is not None else [], dtype=np.int64)
    if nt is None:
        nt = out.n + nsteps
    wav = _f64(wavelets) if wavelets is not None else np.zeros((len(src), nt))
    assert wav.shape == (len(src), nt)
    traces = np.zeros((len(rec), nt))
    rc = lib.orc_run(ctypes.byref(gs), _dp(out.U), _dp(out.Uprev), _aux3(out.Phi), _aux3(out.Psi),
                     out.n, nsteps, len(src), src.ctypes.data_as(_I64P), _dp(wav),
                     len(rec), rec.ctypes.data_as(_I64P), _dp(traces), nt)
    if rc != 0:
        raise MemoryError("oracle run: out of memory")
    out.n += nsteps
    return out, traces


def wave_run(g: Grid, U, Uprev, nsteps: int):
    """Plain leapfrog wave equation with no damping terms (the untruncated
    free-space reference).  Returns (U^{n+k}, U^{n+k-1})."""
    lib = _load()
    gs, keep = g._struct()
    U = _f64(U).copy()
    Up = _f64(Uprev).copy()
    rc = lib.orc_wave_run(ctypes.byref(gs), _dp(U), _dp(Up), nsteps)
    if rc != 0:
        raise MemoryError("oracle wave_run: out of memory")
    return U, Up


def adjoint(g: Grid, U0, nsteps: int, sources, wavelets, receivers, resid):
    """Discrete adjoint of start + ``nsteps`` steps (zero initial velocity)
    for J = 1/2 sum (d - obs)^2, given resid = d - obs of shape [nr][nsteps].
    Returns (dJ/dc2 per cell, dJ/dw of shape [ns][nsteps])."""
    lib = _load()
    gs, keep = g._struct()
    U0 = _f64(U0)
    src = np.ascontiguousarray(sources, dtype=np.int64)
    rec = np.ascontiguousarray(receivers, dtype=np.int64)
    wav = _f64(wavelets)
    res = _f64(resid)
    assert wav.shape == (len(src), nsteps) and res.shape == (len(rec), nsteps)
    gc2 = np.zeros_like(U0)
    gw = np.zeros((len(src), nsteps))
    rc = lib.orc_adjoint(ctypes.byref(gs), _dp(U0), nsteps, len(src), src.ctypes.data_as(_I64P),
                         _dp(wav), len(rec), rec.ctypes.data_as(_I64P), _dp(res), _dp(gc2), _dp(gw))
    if rc != 0:
        raise MemoryError("oracle adjoint: out of memory")
    return gc2, gw


@dataclass
class RKState:
    """First-order state of the RK4 integrator: U, V = U_t, Phi_a, Psi_a."""
    U: np.ndarray
    V: np.ndarray
    Phi: list
    Psi: list
    n: int = 0


def rk4_start(g: Grid, U0, V0=None) -> RKState:
    U0 = _f64(U0).copy()
    V = np.zeros_like(U0) if V0 is None else _f64(V0).copy()
    return RKState(U0, V, [np.zeros_like(U0) for _ in range(g.ndim)],
                   [np.zeros_like(U0) for _ in range(g.ndim)], 0)


def rk4_run(g: Grid, s: RKState, nsteps: int) -> RKState:
    """Classic RK4 on (U, V, Phi, Psi) (the paper's integrator); returns a new state."""
    lib = _load()
    gs, keep = g._struct()
    out = RKState(_f64(s.U).copy(), _f64(s.V).copy(), [_f64(p).copy() for p in s.Phi],
                  [_f64(p).copy() for p in s.Psi], s.n)
    rc = lib.orc_rk4_run(ctypes.byref(gs), _dp(out.U), _dp(out.V), _aux3(out.Phi), _aux3(out.Psi), nsteps)
    if rc != 0:
        raise MemoryError("oracle rk4: out of memory")
    out.n += nsteps
    return out
