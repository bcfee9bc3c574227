"""MI355X (gfx950) stepper for the discrete scalar wave equation with the
reflectionless discrete perfectly matched layer of A. Chern ("A Reflectionless
Discrete Perfectly Matched Layer", arXiv 1804.01390).

This module is a thin ctypes binding over ``libdpml.so`` (C ABI in
``include/dpml.h``): it marshals arguments and uses torch only to allocate
device memory and to name the current HIP stream.  Every step of the scheme
runs in the library's HIP kernels; there is no CPU or torch fallback -- if the
library or the GPU is missing, constructing a ``Simulation`` raises.

Shapes: per-axis sizes are given in the paper's axis order (x, y, z); device
fields are torch tensors of shape reversed(N) (z, y, x), x fastest.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdpml.so")

DPML_OK, DPML_EINVAL, DPML_ENOMEM, DPML_EHIP, DPML_ESTATE, DPML_ENONFINITE = 0, -1, -2, -3, -4, -5
DPML_F32, DPML_F64 = 0, 1
(VARIANT_AUTO, VARIANT_CELL, VARIANT_MARCH, VARIANT_MARCH1, VARIANT_TWOSTEP, VARIANT_THREESTEP,
 VARIANT_FOURSTEP, VARIANT_DEEP) = 0, 1, 2, 3, 4, 5, 6, 7
FIELD_U, FIELD_UPREV = 0, 1


def pass_shape(rows: int = 0, group: int = 0, frame: int = 0, depth: int = 0, ahead: bool = False) -> int:
    """The tile_rows value of a 2D multi-step launch shape: rows per core wave
    (0: 8), rows whose loads a wave issues together (1, 2 or 4; 0: 2), the
    frame form (0 one thread per cell, 1-14 wave marches over spans of that
    many rows, 15 all frame steps of a pass in one launch), the levels per
    pass of VARIANT_DEEP (2-8; 0: 6) and loads issued ahead in cores of four
    or more levels."""
    if not (0 <= rows < 4096 and group in (0, 1, 2, 4) and 0 <= frame <= 15 and depth in (0, 2, 3, 4, 5, 6, 7, 8)):
        raise ValueError("launch shape out of range")
    return rows | (group << 12) | (frame << 16) | (depth << 20) | (int(bool(ahead)) << 24)


def FIELD_PHI(a: int) -> int:
    return 2 + 2 * a


def FIELD_PSI(a: int) -> int:
    return 3 + 2 * a


EXPORTED = [
    "dpml_workspace_bytes", "dpml_create", "dpml_set_state", "dpml_inject", "dpml_record",
    "dpml_record_plane", "dpml_set_variant", "dpml_step", "dpml_step_checked", "dpml_field",
    "dpml_time_index", "dpml_step_graph", "dpml_state_bytes", "dpml_get_state", "dpml_put_state", "dpml_sync",
    "dpml_destroy", "dpml_strerror", "dpml_last_error",
    "dpml_adjoint_workspace_bytes", "dpml_forward_checkpointed", "dpml_adjoint",
    "dpml_multi_workspace_bytes", "dpml_multi_create", "dpml_multi_set_state", "dpml_multi_step",
    "dpml_multi_field", "dpml_multi_tiles", "dpml_multi_set_variant", "dpml_multi_sync", "dpml_multi_destroy",
    "dpml_multi_last_error",
    "dpml_rk4_workspace_bytes", "dpml_rk4_set_state", "dpml_rk4_step", "dpml_rk4_field",
    "dpml_rk4_time_index", "dpml_set_timing", "dpml_get_timing", "dpml_bandwidth_probe",
    "dpml_step_checked_noalloc",
]

PROBE_READ, PROBE_WRITE, PROBE_COPY, PROBE_NONTEMPORAL, PROBE_MAX_BLOCKS = 0, 1, 2, 4, 16384

KERNEL_STEP, KERNEL_PAIR, KERNEL_FRAME, KERNEL_CORE = 0, 1, 2, 3
KERNEL_NAMES = {KERNEL_STEP: "step", KERNEL_PAIR: "pair", KERNEL_FRAME: "frame", KERNEL_CORE: "core"}


class DpmlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("dpml error %d: %s" % (code, msg))
        self.code = code


class TimingT(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4), ("bytes", ctypes.c_double * 4)]


class GridT(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3),
                ("batch", ctypes.c_int64), ("walls", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32)]


_lib = None
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)


def load_library():
    """Load libdpml.so (built by ``python -m paper_1804_01390_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdpml.so is not built; run: python -m paper_1804_01390_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    gp = ctypes.POINTER(GridT)
    sig = {
        "dpml_workspace_bytes": (ctypes.c_size_t, [gp, ctypes.c_int32]),
        "dpml_create": (ctypes.c_int, [gp, ctypes.c_double, ctypes.c_double, _DP, ctypes.c_int64,
                                       _DP * 3, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
        "dpml_set_state": (ctypes.c_int, [_VP, _VP, _VP]),
        "dpml_inject": (ctypes.c_int, [_VP, ctypes.c_int64, _I64P, _VP, ctypes.c_int64]),
        "dpml_record": (ctypes.c_int, [_VP, ctypes.c_int64, _I64P, _VP, ctypes.c_int64]),
        "dpml_record_plane": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _VP, ctypes.c_int64]),
        "dpml_set_variant": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
        "dpml_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
        "dpml_step_checked": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64]),
        "dpml_step_checked_noalloc": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64]),
        "dpml_step_graph": (ctypes.c_int, [_VP, ctypes.c_int64]),
        "dpml_field": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP), ctypes.c_int64 * 3]),
        "dpml_time_index": (ctypes.c_int64, [_VP]),
        "dpml_state_bytes": (ctypes.c_size_t, [_VP]),
        "dpml_get_state": (ctypes.c_int, [_VP, _VP]),
        "dpml_put_state": (ctypes.c_int, [_VP, _VP, ctypes.c_int64]),
        "dpml_sync": (ctypes.c_int, [_VP]),
        "dpml_destroy": (None, [_VP]),
        "dpml_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "dpml_last_error": (ctypes.c_char_p, [_VP]),
        "dpml_adjoint_workspace_bytes": (ctypes.c_size_t, [_VP, ctypes.c_int64, ctypes.c_int64]),
        "dpml_forward_checkpointed": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _VP, ctypes.c_size_t]),
        "dpml_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
        "dpml_multi_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64, gp]),
        "dpml_multi_create": (ctypes.c_int, [ctypes.c_int64, gp, _DP, _DP, ctypes.POINTER(_DP), _VP,
                                             ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
        "dpml_multi_set_state": (ctypes.c_int, [_VP, ctypes.POINTER(_VP)]),
        "dpml_multi_step": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32]),
        "dpml_multi_field": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_VP),
                                            ctypes.c_int64 * 3]),
        "dpml_multi_tiles": (ctypes.c_int64, [_VP]),
        "dpml_multi_set_variant": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "dpml_multi_sync": (ctypes.c_int, [_VP]),
        "dpml_multi_destroy": (None, [_VP]),
        "dpml_multi_last_error": (ctypes.c_char_p, [_VP]),
        "dpml_rk4_workspace_bytes": (ctypes.c_size_t, [_VP]),
        "dpml_rk4_set_state": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP, _VP]),
        "dpml_rk4_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
        "dpml_rk4_field": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP), ctypes.c_int64 * 3]),
        "dpml_rk4_time_index": (ctypes.c_int64, [_VP]),
        "dpml_set_timing": (ctypes.c_int, [_VP, ctypes.c_int32]),
        "dpml_get_timing": (ctypes.c_int, [_VP, ctypes.POINTER(TimingT)]),
        "dpml_bandwidth_probe": (ctypes.c_int, [ctypes.c_int32, _VP, _VP, ctypes.c_size_t, ctypes.c_int32,
                                                ctypes.c_int32, _VP, _DP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _grid(n, lo, hi, dtype_code, batch: int = 1, walls=()) -> GridT:
    g = GridT()
    g.ndim = len(n)
    g.dtype = dtype_code
    g.batch = int(batch)
    for a in range(3):
        g.walls[a] = 1 if (a < len(walls) and walls[a]) else 0
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 1
        g.lo[a] = int(lo[a]) if a < len(n) else 0
        g.hi[a] = int(hi[a]) if a < len(n) else 0
    return g


def workspace_bytes(n, lo, hi, dtype_code: int, c2_field: bool, batch: int = 1) -> int:
    return int(load_library().dpml_workspace_bytes(ctypes.byref(_grid(n, lo, hi, dtype_code, batch)),
                                                   1 if c2_field else 0))


def bandwidth_probe(kind: int, nbytes: int, reps: int = 10, blocks_per_cu: int = 8, buffers=None) -> float:
    """Time the library's streaming probe (PROBE_READ / PROBE_WRITE /
    PROBE_COPY, optionally | PROBE_NONTEMPORAL) over ``nbytes`` bytes on the
    current stream; returns milliseconds per launch.  ``buffers`` = (dst,
    src) device tensors to reuse, else they are allocated here."""
    import torch
    lib = load_library()
    if buffers is None:
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        src.random_(0, 255)
        dst = torch.empty(max(nbytes, PROBE_MAX_BLOCKS * 16), dtype=torch.uint8, device="cuda")
    else:
        dst, src = buffers
    ms = ctypes.c_double(0.0)
    rc = lib.dpml_bandwidth_probe(int(kind), dst.data_ptr(), src.data_ptr(), int(nbytes), int(blocks_per_cu),
                                  int(reps), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  ctypes.byref(ms))
    if rc != DPML_OK:
        raise DpmlError(rc, lib.dpml_strerror(rc).decode())
    return ms.value


class Simulation:
    """One discrete-PML stepper on one GPU.

    n, lo, hi : interior cells and layer cells below/above, per axis (x, y, z)
    h, dt     : grid spacing and time step
    sigma     : per-axis FP64 damping arrays of length lo+n+hi (sigma(i) on
                edge [i, i+1]); None for an undamped axis
    c2        : scalar (1.0) or FP64 array of shape reversed(N)
    dtype     : torch.float32 or torch.float64
    batch     : independent problems (shots) sharing c2 and sigma; fields are
                then [batch, *reversed(N)] and cell indices address the batch
    walls     : per axis, True for reflecting walls instead of periodic wrap
    """

    def __init__(self, n: Sequence[int], lo: Sequence[int], hi: Sequence[int], h: float, dt: float,
                 sigma: Sequence[Optional[np.ndarray]], c2=1.0, dtype=None, device=None,
                 batch: int = 1, walls=()):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1804_01390_amd needs a ROCm GPU; none is visible")
        self.torch = torch
        self.lib = load_library()
        self.dtype = dtype if dtype is not None else torch.float32
        if self.dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.code = DPML_F32 if self.dtype == torch.float32 else DPML_F64
        self.device = torch.device(device if device is not None else "cuda:0")
        self.n, self.lo, self.hi = list(n), list(lo), list(hi)
        self.ndim = len(n)
        self.N = [self.lo[a] + self.n[a] + self.hi[a] for a in range(self.ndim)]
        self.batch = int(batch)
        self.member_shape = tuple(reversed(self.N))
        self.shape = self.member_shape if self.batch == 1 else (self.batch,) + self.member_shape
        self.cells = int(np.prod(self.N))
        self.h, self.dt = float(h), float(dt)
        c2a = np.ascontiguousarray(np.asarray(c2, dtype=np.float64).reshape(-1))
        field = c2a.size != 1
        self.walls = tuple(bool(w) for w in walls)
        g = _grid(self.n, self.lo, self.hi, self.code, self.batch, self.walls)
        nbytes = self.lib.dpml_workspace_bytes(ctypes.byref(g), 1 if field else 0)
        if nbytes == 0:
            raise DpmlError(DPML_EINVAL, "invalid grid")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        sig3 = (_DP * 3)()
        self._sig_keep = []
        for a in range(3):
            if a < self.ndim and sigma is not None and a < len(sigma) and sigma[a] is not None:
                s = np.ascontiguousarray(np.asarray(sigma[a], dtype=np.float64))
                if s.shape != (self.N[a],):
                    raise ValueError("sigma[%d] must have %d entries" % (a, self.N[a]))
                self._sig_keep.append(s)
                sig3[a] = s.ctypes.data_as(_DP)
            else:
                sig3[a] = _DP()
        handle = _VP()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = self.lib.dpml_create(ctypes.byref(g), self.h, self.dt, c2a.ctypes.data_as(_DP), c2a.size,
                                  sig3, ctypes.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                  ctypes.c_void_p(stream), ctypes.byref(handle))
        if rc != DPML_OK:
            raise DpmlError(rc, self.lib.dpml_last_error(None).decode())
        self.handle = handle
        self._keep = {}

    # -- helpers ----------------------------------------------------------
    def _check(self, rc: int):
        if rc != DPML_OK:
            raise DpmlError(rc, self.lib.dpml_last_error(self.handle).decode())

    def _dev(self, t):
        t = self.torch.as_tensor(t)
        if t.device != self.device or t.dtype != self.dtype or not t.is_contiguous():
            t = t.to(device=self.device, dtype=self.dtype).contiguous()
        return t

    # -- API ----------------------------------------------------------------
    def set_variant(self, variant: int, tile_rows: int = 0):
        """Kernel variant (VARIANT_*) and its launch shape (0: defaults; for
        the multi-step variants see ``pass_shape``).  Results do not depend on
        the choice; ``autotune.tune`` picks the fastest."""
        self._check(self.lib.dpml_set_variant(self.handle, variant, tile_rows))

    def set_state(self, U0, V0=None):
        """U^0 (and optional V^0) as arrays/tensors of shape reversed(N)."""
        U0 = self._dev(U0)
        if tuple(U0.shape) != self.shape:
            raise ValueError("U0 must have shape %s" % (self.shape,))
        V = None if V0 is None else self._dev(V0)
        self._keep["U0"], self._keep["V0"] = U0, V
        self._check(self.lib.dpml_set_state(self.handle, ctypes.c_void_p(U0.data_ptr()),
                                            ctypes.c_void_p(V.data_ptr() if V is not None else 0)))

    def inject(self, cells: Sequence[int], wavelets):
        """Point sources at flat cell indices with wavelets [ns][nt]."""
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1))
        w = self._dev(wavelets)
        if w.dim() != 2 or w.shape[0] != c.size:
            raise ValueError("wavelets must be [ns][nt]")
        self._keep["wavelets"] = w
        self._check(self.lib.dpml_inject(self.handle, c.size, c.ctypes.data_as(_I64P),
                                         ctypes.c_void_p(w.data_ptr()), w.shape[1]))

    def record(self, cells: Sequence[int], nt: int):
        """Point receivers; returns the device trace tensor [nr][nt]."""
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1))
        tr = self.torch.zeros((c.size, nt), dtype=self.dtype, device=self.device)
        self._keep["traces"] = tr
        self._check(self.lib.dpml_record(self.handle, c.size, c.ctypes.data_as(_I64P),
                                         ctypes.c_void_p(tr.data_ptr()), nt))
        return tr

    def record_plane(self, axis: int, index: int, nt: int):
        """Record U on the plane i_axis = index after every step; returns the
        device tensor [nt][...] (remaining axes, slowest first)."""
        rest = [self.N[a] for a in range(self.ndim) if a != axis]
        pl = self.torch.zeros([nt] + list(reversed(rest)), dtype=self.dtype, device=self.device)
        self._keep["planes"] = pl
        self._check(self.lib.dpml_record_plane(self.handle, axis, index, ctypes.c_void_p(pl.data_ptr()), nt))
        return pl

    def step(self, nsteps: int = 1):
        self._check(self.lib.dpml_step(self.handle, int(nsteps)))

    def step_graph(self, nsteps: int):
        """nsteps steps replayed from a cached HIP graph (no sources/receivers)."""
        self._check(self.lib.dpml_step_graph(self.handle, int(nsteps)))

    def step_checked(self, nsteps: int, every: int):
        self._check(self.lib.dpml_step_checked(self.handle, int(nsteps), int(every)))

    def step_checked_noalloc(self, nsteps: int, every: int):
        """As step_checked, through the entry point that allocates nothing
        (one thread per cell, scan flags in the library's static array)."""
        self._check(self.lib.dpml_step_checked_noalloc(self.handle, int(nsteps), int(every)))

    def field(self, which: int):
        """Borrowed view of a field of the current level (valid until the next step)."""
        ptr = _VP()
        shape = (ctypes.c_int64 * 3)()
        self._check(self.lib.dpml_field(self.handle, which, ctypes.byref(ptr), shape))
        ext = [shape[a] for a in range(self.ndim)]
        off = ptr.value - self.workspace.data_ptr()
        esize = 4 if self.code == DPML_F32 else 8
        count = int(np.prod(ext)) * self.batch
        raw = self.workspace[off: off + count * esize]
        view = tuple(reversed(ext)) if self.batch == 1 else (self.batch,) + tuple(reversed(ext))
        return raw.view(self.dtype).view(view)

    @property
    def U(self):
        return self.field(FIELD_U)

    @property
    def time_index(self) -> int:
        return int(self.lib.dpml_time_index(self.handle))

    def get_state(self):
        nb = int(self.lib.dpml_state_bytes(self.handle))
        blob = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.dpml_get_state(self.handle, ctypes.c_void_p(blob.data_ptr())))
        return blob, self.time_index

    def put_state(self, blob, n: int):
        self._check(self.lib.dpml_put_state(self.handle, ctypes.c_void_p(blob.data_ptr()), int(n)))

    def sync(self):
        self._check(self.lib.dpml_sync(self.handle))

    def set_timing(self, enable: bool = True):
        """Bracket each step-kernel launch with HIP events on the handle's stream."""
        self._check(self.lib.dpml_set_timing(self.handle, 1 if enable else 0))

    def get_timing(self):
        """Per kernel class ("step", "pair", "frame", "core"): launches, summed milliseconds
        and summed algorithmic bytes of the launches since timing was enabled."""
        t = TimingT()
        self._check(self.lib.dpml_get_timing(self.handle, ctypes.byref(t)))
        return {KERNEL_NAMES[k]: {"launches": int(t.launches[k]), "ms": float(t.ms[k]), "bytes": float(t.bytes[k])}
                for k in KERNEL_NAMES if t.launches[k] > 0}

    # -- RK4 (the paper's integrator) -----------------------------------------
    def rk4_set_state(self, U0, V0=None):
        nb = int(self.lib.dpml_rk4_workspace_bytes(self.handle))
        if nb == 0:
            raise DpmlError(DPML_EINVAL, "RK4 needs batch == 1")
        if self._keep.get("rk_ws") is None or self._keep["rk_ws"].numel() < nb:
            self._keep["rk_ws"] = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        ws = self._keep["rk_ws"]
        U0 = self._dev(U0)
        V = None if V0 is None else self._dev(V0)
        self._keep["rk_U0"], self._keep["rk_V0"] = U0, V
        self._check(self.lib.dpml_rk4_set_state(self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                                ctypes.c_void_p(U0.data_ptr()),
                                                ctypes.c_void_p(V.data_ptr() if V is not None else 0)))

    def rk4_step(self, nsteps: int = 1):
        self._check(self.lib.dpml_rk4_step(self.handle, int(nsteps)))

    def rk4_field(self, which: int):
        ptr = _VP()
        shape = (ctypes.c_int64 * 3)()
        self._check(self.lib.dpml_rk4_field(self.handle, which, ctypes.byref(ptr), shape))
        ext = [shape[a] for a in range(self.ndim)]
        ws = self._keep["rk_ws"]
        off = ptr.value - ws.data_ptr()
        esize = 4 if self.code == DPML_F32 else 8
        count = int(np.prod(ext))
        return ws[off: off + count * esize].view(self.dtype).view(tuple(reversed(ext)))

    # -- adjoint --------------------------------------------------------------
    def forward_checkpointed(self, nsteps: int, ckpt_every: int = 0):
        """Run nsteps from time 0 saving sqrt(T) checkpoints (or every
        ``ckpt_every`` steps) for a later ``adjoint`` call."""
        every = int(ckpt_every) if ckpt_every > 0 else max(1, int(round(math.sqrt(nsteps))))
        nb = int(self.lib.dpml_adjoint_workspace_bytes(self.handle, int(nsteps), every))
        if nb == 0:
            raise DpmlError(DPML_EINVAL, "bad checkpoint arguments")
        if self._keep.get("adj_ws") is None or self._keep["adj_ws"].numel() < nb:
            self._keep["adj_ws"] = None
            self._keep["adj_ws"] = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        ws = self._keep["adj_ws"]
        self._check(self.lib.dpml_forward_checkpointed(self.handle, int(nsteps), every,
                                                       ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        self.adj_nsteps = int(nsteps)

    def adjoint(self, resid, grad_c2=None, want_wavelets: bool = True):
        """Gradients for J = 1/2 sum (traces - obs)^2 given resid = traces - obs
        ([nr][nt], same layout as the trace buffer).  Returns (dJ/dc2 as FP64
        tensor of one member's shape, dJ/dw [ns][nt] or None)."""
        res = self._dev(resid) if resid is not None else None
        if grad_c2 is None:
            grad_c2 = self.torch.zeros(self.member_shape, dtype=self.torch.float64, device=self.device)
        gw = None
        if want_wavelets and "wavelets" in self._keep:
            gw = self.torch.zeros_like(self._keep["wavelets"])
        self._check(self.lib.dpml_adjoint(self.handle, ctypes.c_void_p(res.data_ptr() if res is not None else 0),
                                          ctypes.c_void_p(grad_c2.data_ptr()),
                                          ctypes.c_void_p(gw.data_ptr() if gw is not None else 0)))
        self._keep["resid"] = res
        return grad_c2, gw

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dpml_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiSimulation:
    """Many independent 2D problems of different sizes advanced together by
    one kernel launch per step (optionally one HIP-graph launch per run).

    problems: sequence of objects with attributes n, lo, hi (2 entries each),
              h, dt and sigma (two FP64 arrays); unit wave speed.
    """

    def __init__(self, problems, dtype=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1804_01390_amd needs a ROCm GPU; none is visible")
        self.torch = torch
        self.lib = load_library()
        self.dtype = dtype if dtype is not None else torch.float32
        self.code = DPML_F32 if self.dtype == torch.float32 else DPML_F64
        self.device = torch.device(device if device is not None else "cuda:0")
        self.count = len(problems)
        grids = (GridT * self.count)()
        h = np.ascontiguousarray([float(p.h) for p in problems])
        dt = np.ascontiguousarray([float(p.dt) for p in problems])
        sig = (_DP * (3 * self.count))()
        self._keep_host = []
        self.shapes = []
        for i, p in enumerate(problems):
            grids[i] = _grid(p.n, p.lo, p.hi, self.code)
            N = [p.lo[a] + p.n[a] + p.hi[a] for a in range(2)]
            self.shapes.append(tuple(reversed(N)))
            for a in range(3):
                if a < 2 and p.sigma[a] is not None:
                    arr = np.ascontiguousarray(p.sigma[a], dtype=np.float64)
                    self._keep_host.append(arr)
                    sig[3 * i + a] = arr.ctypes.data_as(_DP)
                else:
                    sig[3 * i + a] = _DP()
        nbytes = self.lib.dpml_multi_workspace_bytes(self.count, grids)
        if nbytes == 0:
            raise DpmlError(DPML_EINVAL, self.lib.dpml_multi_last_error(None).decode())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
        handle = _VP()
        rc = self.lib.dpml_multi_create(self.count, grids, h.ctypes.data_as(_DP), dt.ctypes.data_as(_DP),
                                        sig, ctypes.c_void_p(self.workspace.data_ptr()), int(nbytes),
                                        ctypes.c_void_p(stream), ctypes.byref(handle))
        if rc != DPML_OK:
            raise DpmlError(rc, self.lib.dpml_multi_last_error(None).decode())
        self.handle = handle
        self.tiles = int(self.lib.dpml_multi_tiles(handle))
        self.cells = int(sum(int(np.prod(s)) for s in self.shapes))
        self._keep = []

    def _check(self, rc):
        if rc != DPML_OK:
            raise DpmlError(rc, self.lib.dpml_multi_last_error(self.handle).decode())

    def set_state(self, U0s):
        ts = []
        for i, u in enumerate(U0s):
            t = self.torch.as_tensor(u).to(device=self.device, dtype=self.dtype).contiguous()
            if tuple(t.shape) != self.shapes[i]:
                raise ValueError("U0[%d] must have shape %s" % (i, self.shapes[i]))
            ts.append(t)
        ptrs = (_VP * self.count)(*[t.data_ptr() for t in ts])
        self._keep = ts
        self._check(self.lib.dpml_multi_set_state(self.handle, ptrs))

    def step(self, nsteps: int, graph: bool = False):
        self._check(self.lib.dpml_multi_step(self.handle, int(nsteps), 1 if graph else 0))

    def set_variant(self, variant: int = 0, tile_rows: int = 0, group: int = 0):
        """Stepping scheme (VARIANT_MARCH single steps, VARIANT_TWOSTEP,
        THREESTEP, FOURSTEP or DEEP multi-step passes; DEEP takes its depth
        in bits 20-23 of tile_rows) and its tile height and
        row-load group (0: defaults); results do not depend on them."""
        self._check(self.lib.dpml_multi_set_variant(self.handle, int(variant), int(tile_rows), int(group)))
        self.tiles = int(self.lib.dpml_multi_tiles(self.handle))
        self.launch = (int(variant), int(tile_rows), int(group))

    def field(self, prob: int, which: int):
        ptr = _VP()
        shape = (ctypes.c_int64 * 3)()
        self._check(self.lib.dpml_multi_field(self.handle, prob, which, ctypes.byref(ptr), shape))
        ext = [shape[0], shape[1]]
        off = ptr.value - self.workspace.data_ptr()
        esize = 4 if self.code == DPML_F32 else 8
        count = ext[0] * ext[1]
        return self.workspace[off: off + count * esize].view(self.dtype).view(ext[1], ext[0])

    def sync(self):
        self._check(self.lib.dpml_multi_sync(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dpml_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
