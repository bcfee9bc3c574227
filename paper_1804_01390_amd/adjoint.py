"""torch.autograd interface to the library's discrete adjoint.

``receiver_traces(problem, c2, wavelets)`` runs a batch of shots (one
Simulation of ``batch`` members sharing c^2) and returns the receiver traces
``[batch, nr, nt]``; its backward runs the hand-written reverse-time adjoint
kernel (sqrt(T) checkpointing, FP64 accumulation of dJ/dc^2 over shots and
steps) and returns the vector-Jacobian products for c^2 and the wavelets.
The forward and the adjoint both run in the HIP library; torch only holds
memory and chains the gradients.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import Simulation


@dataclass
class ShotProblem:
    """A batch of shots on one grid (x, y[, z] order per axis).

    sources[b]   flat cell indices (within one member) of shot b's sources
    receivers    flat cell indices (within one member) shared by all shots
    """
    n: Sequence[int]
    lo: Sequence[int]
    hi: Sequence[int]
    h: float
    dt: float
    sigma: Sequence[Optional[np.ndarray]]
    sources: List[List[int]]
    receivers: List[int]
    nt: int
    dtype: torch.dtype = torch.float32
    ckpt_every: int = 0
    U0: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return len(self.sources)

    @property
    def cells(self) -> int:
        return int(np.prod([self.lo[a] + self.n[a] + self.hi[a] for a in range(len(self.n))]))


class _TracesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c2: torch.Tensor, wavelets: torch.Tensor, prob: ShotProblem):
        c2_host = c2.detach().to("cpu", torch.float64).numpy()
        sim = Simulation(prob.n, prob.lo, prob.hi, prob.h, prob.dt, prob.sigma, c2=c2_host,
                         dtype=prob.dtype, batch=prob.batch)
        B, cells = prob.batch, prob.cells
        if prob.U0 is None:
            U0 = torch.zeros(sim.shape, dtype=prob.dtype, device=sim.device)
        else:
            U0 = torch.as_tensor(prob.U0)
        sim.set_state(U0)
        src = [b * cells + c for b in range(B) for c in prob.sources[b]]
        w = wavelets.detach().to(sim.device, prob.dtype).reshape(len(src), prob.nt).contiguous()
        sim.inject(src, w)
        rec = [b * cells + c for b in range(B) for c in prob.receivers]
        tr = sim.record(rec, prob.nt)
        sim.forward_checkpointed(prob.nt, prob.ckpt_every)
        ctx.sim = sim
        ctx.c2_dtype = c2.dtype
        ctx.c2_device = c2.device
        ctx.w_shape = wavelets.shape
        ctx.w_dtype = wavelets.dtype
        ctx.w_device = wavelets.device
        return tr.view(B, len(prob.receivers), prob.nt).clone()

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        sim = ctx.sim
        resid = grad_traces.reshape(-1, grad_traces.shape[-1]).contiguous()
        gc2, gw = sim.adjoint(resid)
        sim.sync()
        gc2 = gc2.to(ctx.c2_device, ctx.c2_dtype)
        gw = gw.reshape(ctx.w_shape).to(ctx.w_device, ctx.w_dtype) if gw is not None else None
        ctx.sim = None
        sim.close()
        return gc2, gw, None


def receiver_traces(prob: ShotProblem, c2: torch.Tensor, wavelets: torch.Tensor) -> torch.Tensor:
    """Traces [batch, nr, nt] of the shots in ``prob`` for wave-speed field
    ``c2`` (shape of one member, FP64 or FP32) and ``wavelets``
    [total sources, nt]; differentiable in c2 and wavelets."""
    return _TracesFn.apply(c2, wavelets, prob)
