"""Velocity gradient through torch.autograd (argument marshalling only).

``FWIGradient.apply(vel, problem)`` runs the forward propagation in libfd
with wavefield checkpoints every ``problem.ckpt_every`` steps and returns the
receiver traces.  Its backward runs libfd's adjoint propagation with segment
recomputation and the fused zero-lag imaging condition, then the velocity
chain rule, and returns dJ/dv for whatever scalar J autograd differentiates
(the trace cotangent is the adjoint source).  All arithmetic happens in the
library's kernels; this module only allocates caller-owned device buffers.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import fd as FD


@dataclass
class ShotProblem:
    """One shot on one grid: geometry, wavelet and checkpoint interval."""
    shape: tuple
    spacing: tuple
    so: int
    dt: float
    vmax: float
    nbl: int
    nt: int
    src: np.ndarray          # [ns][ndim] metres
    rec: np.ndarray          # [nr][ndim] metres
    q: np.ndarray            # [nt][ns] float32
    ckpt_every: int = 50
    boundary: int = FD.FD_BC_ZERO
    device: int = 0


class FWIGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel: torch.Tensor, pb: ShotProblem):
        g = FD.Grid(pb.shape, pb.spacing, pb.so, pb.dt, pb.vmax, nbl=pb.nbl,
                    boundary=pb.boundary, device=pb.device)
        g.set_model(vel.detach().contiguous())
        S, R = g.sparse(pb.src), g.sparse(pb.rec)
        q = torch.as_tensor(pb.q, dtype=torch.float32, device=vel.device).contiguous()
        k = max(1, min(pb.ckpt_every, pb.nt))
        nck = (pb.nt + k - 1) // k
        ckpt = [g.field() for _ in range(2 * nck)]
        d = torch.zeros((pb.nt, R.n), dtype=torch.float32, device=vel.device)
        g.forward([g.field(), g.field()], S, q, R, d, pb.nt, ckpt=ckpt, ckpt_every=k)
        ctx.g, ctx.S, ctx.R, ctx.q, ctx.ckpt, ctx.k, ctx.nt = g, S, R, q, ckpt, k, pb.nt
        ctx.vshape = vel.shape
        return d

    @staticmethod
    def backward(ctx, grad_d: torch.Tensor):
        g = ctx.g
        dev = grad_d.device
        slots = [g.field() for _ in range(ctx.k + 2)]
        gm = torch.zeros(ctx.vshape, dtype=torch.float32, device=dev)
        g.adjoint([g.field(), g.field()], ctx.R, grad_d.contiguous().float(), ctx.S, ctx.q, None,
                  ctx.nt, ckpt=ctx.ckpt, ckpt_every=ctx.k, slots=slots, grad_m=gm)
        gv = torch.empty_like(gm)
        g.gradient_to_velocity(gm, gv)
        ctx.ckpt = None
        return gv, None


def fwi_gradient(vel: torch.Tensor, pb: ShotProblem, d_obs: torch.Tensor):
    """(J, dJ/dv) for J = 1/2 |d(v) - d_obs|^2."""
    v = vel.detach().requires_grad_(True)
    d = FWIGradient.apply(v, pb)
    J = 0.5 * torch.sum((d - d_obs) ** 2)
    J.backward()
    return J.detach(), v.grad
