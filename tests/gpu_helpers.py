"""Shared helpers for the GPU parity tests: run one workload through the HIP
library (via the C ABI binding) and through the FP64 oracle on the same
seeded inputs."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2312_13094_amd import fd as FD


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def wrapped_boxes(g, f, names, pt, w):
    """The DOMAIN values of fields f (named by names) on the box of
    half-width w around pt, at periodically wrapped indices, as float64."""
    import torch
    idx = [torch.from_numpy(np.arange(int(k) - w, int(k) + w + 1) % n).cuda()
           for k, n in zip(pt, g.shape)]
    return {name: g.domain(t).index_select(0, idx[0]).index_select(1, idx[1])
            .index_select(2, idx[2]).double().cpu().numpy() for name, t in zip(names, f)}


def gpu_grid(shape, spacing, so, dt, vmax, nbl=0, boundary=FD.FD_BC_ZERO, tile=None):
    g = FD.Grid(shape, spacing, so, dt, vmax, nbl=nbl, boundary=boundary)
    if tile is not None:
        g.set_tile(*tile)
    return g


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_gpu_forward(shape, spacing, so, dt, vmax, v, nt, nbl=0, boundary=0, src=None, q=None,
                    rec=None, u0=None, um=None, tile=None):
    """Returns (u^nt DOMAIN, u^(nt-1) DOMAIN, traces) as float64 numpy."""
    import torch
    g = gpu_grid(shape, spacing, so, dt, vmax, nbl, boundary, tile)
    g.set_model(to_dev(np.asarray(v, dtype=np.float32)))
    a, b = g.field(), g.field()
    if u0 is not None:
        g.domain(a).copy_(to_dev(np.asarray(u0, dtype=np.float32)))
    if um is not None:
        g.domain(b).copy_(to_dev(np.asarray(um, dtype=np.float32)))
    S = g.sparse(src) if src is not None else None
    R = g.sparse(rec) if rec is not None else None
    qd = to_dev(np.asarray(q, dtype=np.float32)) if S is not None else None
    d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda") if R is not None else None
    g.forward([a, b], S, qd, R, d, nt)
    torch.cuda.synchronize()
    out = (g.domain(a).double().cpu().numpy(), g.domain(b).double().cpu().numpy(),
           None if d is None else d.double().cpu().numpy())
    g.close()
    return out


def run_oracle_forward(shape, spacing, so, dt, vmax, v, nt, nbl=0, boundary=0, src=None, q=None,
                       rec=None, u0=None, um=None):
    g = O.Grid(tuple(shape), tuple(spacing), so=so, dt=dt, nbl=nbl, vmax=vmax, bc=boundary)
    v64 = np.asarray(v, dtype=np.float32).astype(np.float64)
    a = g.pad(np.asarray(u0, dtype=np.float32).astype(np.float64)) if u0 is not None else None
    b = g.pad(np.asarray(um, dtype=np.float32).astype(np.float64)) if um is not None else None
    qq = None if q is None else np.asarray(q, dtype=np.float32).astype(np.float64)
    u, uo, d, _ = O.forward(g, v64, src, qq, rec, nt, u0=a, um=b)
    return g.interior(u), g.interior(uo), d
