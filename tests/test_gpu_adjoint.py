"""GPU adjoint propagation and checkpointed imaging gradient against the FP64
oracle, and the FP32 dot-product test."""
import numpy as np
import pytest

import oracle as O
from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _fd():
    from paper_2312_13094_amd import fd
    return fd


def _setup(shape, so, nbl, bc, seed, nsrc=2, nrec=25, vlo=1500.0, vhi=3500.0):
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    h = 10.0
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), vlo, vhi).astype(np.float32)
    dt = synth.stable_dt(so, ndim, h, vhi)
    src = np.stack([rng.uniform(h, (s - 2) * h, nsrc) for s in shape], 1)
    rec = np.stack([rng.uniform(h, (s - 2) * h, nrec) for s in shape], 1)
    return rng, dict(shape=shape, spacing=(h,) * ndim, so=so, dt=dt, vmax=vhi, nbl=nbl, bc=bc,
                     v=v, src=src, rec=rec)


def _grid(c):
    FD = _fd()
    g = FD.Grid(c["shape"], c["spacing"], c["so"], c["dt"], c["vmax"], nbl=c["nbl"],
                boundary=c["bc"])
    g.set_model(to_dev(c["v"]))
    return g


def _gpu_fwd(g, S, R, q, nt, ckpt=None, k=0):
    import torch
    a, b = g.field(), g.field()
    d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda")
    g.forward([a, b], S, to_dev(q), R, d, nt, ckpt=ckpt, ckpt_every=k)
    return d


def _gpu_adj(g, S, R, resid, nt, q=None, ckpt=None, k=0, grad=False):
    import torch
    a, b = g.field(), g.field()
    qa = torch.zeros((nt, S.n), dtype=torch.float32, device="cuda")
    gm = torch.zeros(g.shape, dtype=torch.float32, device="cuda") if grad else None
    slots = [g.field() for _ in range(k + 2)] if grad else None
    g.adjoint([a, b], R, to_dev(resid), S, None if q is None else to_dev(q), qa, nt,
              ckpt=ckpt, ckpt_every=k, slots=slots, grad_m=gm)
    torch.cuda.synchronize()
    return qa, gm, (a, b)


@pytest.mark.parametrize("shape,so,nbl,bc", [((60, 54), 4, 10, 0), ((26, 30, 70), 8, 5, 0),
                                           ((28, 24, 66), 8, 6, 1), ((40, 44), 12, 8, 1)])
def test_dot_product_fp32(shape, so, nbl, bc):
    rng, c = _setup(shape, so, nbl, bc, 21)
    nt = 60
    g = _grid(c)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    q = rng.standard_normal((nt, S.n)).astype(np.float32)
    r = rng.standard_normal((nt, R.n)).astype(np.float32)
    d = _gpu_fwd(g, S, R, q, nt).double().cpu().numpy()
    qa, _, _ = _gpu_adj(g, S, R, r, nt)
    qa = qa.double().cpu().numpy()
    lhs, rhs = np.sum(d * r.astype(np.float64)), np.sum(q.astype(np.float64) * qa)
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs)), (lhs, rhs)
    g.close()


@pytest.mark.parametrize("shape,so,nbl,bc", [((50, 46), 8, 8, 0), ((22, 26, 68), 8, 5, 1)])
def test_adjoint_matches_oracle(shape, so, nbl, bc):
    rng, c = _setup(shape, so, nbl, bc, 22)
    nt = 80
    g = _grid(c)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    r = rng.standard_normal((nt, R.n)).astype(np.float32)
    qa, _, (l0, l1) = _gpu_adj(g, S, R, r, nt)
    og = O.Grid(shape, c["spacing"], so=so, dt=c["dt"], nbl=nbl, vmax=c["vmax"], bc=bc)
    lam0, lam1, oqa, _ = O.adjoint(og, c["v"].astype(np.float64), c["rec"], r.astype(np.float64),
                                   c["src"], nt)
    assert rel_l2(qa.double().cpu().numpy(), oqa) <= 1e-4
    assert rel_l2(g.domain(l0).double().cpu().numpy(), og.interior(lam0)) <= 1e-4
    assert rel_l2(g.domain(l1).double().cpu().numpy(), og.interior(lam1)) <= 1e-4
    g.close()


@pytest.mark.parametrize("shape,so,nbl,bc,nt,k", [((48, 52), 4, 8, 0, 90, 7),
                                                ((24, 28, 66), 8, 5, 0, 70, 16),
                                                ((26, 24, 64), 8, 5, 1, 50, 50),
                                                ((20, 22, 70), 8, 0, 0, 60, 11),
                                                ((40, 130), 4, 0, 1, 60, 9)])
def test_gradient_matches_oracle(shape, so, nbl, bc, nt, k):
    """Checkpoint every k steps (k need not divide nt), recompute each segment
    into k+2 slots, imaging condition fused into the adjoint sweep; FP32
    gradient vs the FP64 oracle's (which stores every forward state)."""
    import torch
    rng, c = _setup(shape, so, nbl, bc, 23, nsrc=1, nrec=30, vlo=1800.0, vhi=2600.0)
    g = _grid(c)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    q = (synth.ricker(nt, c["dt"], 20.0)[:, None] * 1e3).astype(np.float32)
    # observed data from a perturbed model, computed by the oracle
    og = O.Grid(shape, c["spacing"], so=so, dt=c["dt"], nbl=nbl, vmax=c["vmax"], bc=bc)
    vt = c["v"].astype(np.float64) * 1.03
    _, _, dobs, _ = O.forward(og, vt, c["src"], q.astype(np.float64), c["rec"], nt)
    og0 = O.Grid(shape, c["spacing"], so=so, dt=c["dt"], nbl=nbl, vmax=c["vmax"], bc=bc)
    v64 = c["v"].astype(np.float64)
    _, _, od, hist = O.forward(og0, v64, c["src"], q.astype(np.float64), c["rec"], nt,
                               history=True)
    resid = (od - dobs).astype(np.float32)      # the same residual drives both sides
    _, _, _, ogm = O.adjoint(og0, v64, c["rec"], resid.astype(np.float64), c["src"], nt,
                             hist=hist)
    nck = (nt + k - 1) // k
    ckpt = [g.field() for _ in range(2 * nck)]
    d = _gpu_fwd(g, S, R, q, nt, ckpt=ckpt, k=k)
    assert rel_l2(d.double().cpu().numpy(), od) <= 1e-4
    _, gm, _ = _gpu_adj(g, S, R, resid, nt, q=q, ckpt=ckpt, k=k, grad=True)
    assert rel_l2(gm.double().cpu().numpy(), ogm) <= 1e-3
    # velocity chain rule in the library
    gv = torch.zeros_like(gm)
    g.gradient_to_velocity(gm, gv)
    torch.cuda.synchronize()
    assert rel_l2(gv.double().cpu().numpy(), ogm * (-2.0 / v64 ** 3)) <= 1e-3
    g.close()


def test_gradient_independent_of_checkpoint_interval():
    """Same single-source gradient for k = 5, 13 and one segment (bit-exact:
    recomputation replays the identical kernels)."""
    rng, c = _setup((40, 36, 64), 8, 5, 0, 24, nsrc=1, nrec=20)
    nt = 39
    g = _grid(c)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    q = (synth.ricker(nt, c["dt"], 20.0)[:, None] * 1e3).astype(np.float32)
    r = rng.standard_normal((nt, R.n)).astype(np.float32)
    out = []
    for k in (5, 13, nt):
        ckpt = [g.field() for _ in range(2 * ((nt + k - 1) // k))]
        _gpu_fwd(g, S, R, q, nt, ckpt=ckpt, k=k)
        _, gm, _ = _gpu_adj(g, S, R, r, nt, q=q, ckpt=ckpt, k=k, grad=True)
        out.append(gm.cpu().numpy())
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[0], out[2])
    g.close()


def test_gradient_requires_checkpoints():
    FD = _fd()
    _, c = _setup((20, 20, 20), 4, 2, 0, 25)
    g = _grid(c)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    import torch
    gm = torch.zeros(g.shape, device="cuda")
    r = torch.zeros((10, R.n), device="cuda")
    with pytest.raises(FD.FdError):
        g.adjoint([g.field(), g.field()], R, r, S, None, None, 10, grad_m=gm)
    g.close()


def test_autograd_function_returns_velocity_gradient():
    """FWIGradient (torch.autograd.Function over fd_forward / fd_adjoint) gives
    dJ/dv of J = 1/2 |d - d_obs|^2 matching the FP64 oracle's."""
    import torch
    from paper_2312_13094_amd.fwi import ShotProblem, fwi_gradient
    rng, c = _setup((28, 30, 64), 8, 5, 0, 26, nsrc=1, nrec=30, vlo=1800.0, vhi=2600.0)
    nt = 60
    q = (synth.ricker(nt, c["dt"], 20.0)[:, None] * 1e3).astype(np.float32)
    og = O.Grid(c["shape"], c["spacing"], so=8, dt=c["dt"], nbl=5, vmax=c["vmax"], bc=0)
    v64 = c["v"].astype(np.float64)
    _, _, dobs, _ = O.forward(og, v64 * 1.02, c["src"], q.astype(np.float64), c["rec"], nt)
    _, _, od, hist = O.forward(og, v64, c["src"], q.astype(np.float64), c["rec"], nt, history=True)
    _, _, _, ogm = O.adjoint(og, v64, c["rec"], od - dobs, c["src"], nt, hist=hist)
    ogv = ogm * (-2.0 / v64 ** 3)
    pb = ShotProblem(c["shape"], c["spacing"], 8, c["dt"], c["vmax"], 5, nt, c["src"], c["rec"], q,
                     ckpt_every=11)
    J, gv = fwi_gradient(to_dev(c["v"]), pb, to_dev(dobs.astype(np.float32)))
    torch.cuda.synchronize()
    assert abs(J.item() - 0.5 * np.sum((od - dobs) ** 2)) <= 1e-3 * 0.5 * np.sum((od - dobs) ** 2)
    assert rel_l2(gv.double().cpu().numpy(), ogv) <= 2e-3


@pytest.mark.parametrize("shape,bc,tile", [((40, 36, 70), 1, None), ((40, 36, 70), 0, (4, 2, 16, 12)),
                                           ((30, 34, 66), 1, (4, 4, 8, 4))])
def test_twelve_thousand_receivers_forward_and_adjoint(shape, bc, tile):
    """12,000 receivers scattered through a 3-D grid and 3 sources.  Forward:
    the traces, sampled either inside the step kernel across its blocks (ring
    tiles) or by the multi-block sampler, within 1e-4 of the oracle.
    Adjoint: the receivers inject 12,000 residual traces (multi-block
    injection with float atomics, then multi-block sampling of the sources):
    lambda_0, lambda_1 and the source-side traces within 1e-4."""
    rng, c = _setup(shape, 8, 5, bc, 91, nsrc=3, nrec=12000)
    nt = 24
    g = _grid(c)
    if tile is not None:
        g.set_tile(*tile)
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    q = (synth.ricker(nt, c["dt"], 30.0)[:, None] * np.array([1e3, -7e2, 4e2])).astype(np.float32)
    d = _gpu_fwd(g, S, R, q, nt).double().cpu().numpy()
    og = O.Grid(shape, c["spacing"], so=8, dt=c["dt"], nbl=5, vmax=c["vmax"], bc=bc)
    v64 = c["v"].astype(np.float64)
    _, _, od, _ = O.forward(og, v64, c["src"], q.astype(np.float64), c["rec"], nt)
    assert np.abs(od).max() > 0
    assert rel_l2(d, od) <= 1e-4
    r = rng.standard_normal((nt, R.n)).astype(np.float32)
    qa, _, (l0, l1) = _gpu_adj(g, S, R, r, nt)
    lam0, lam1, oqa, _ = O.adjoint(og, v64, c["rec"], r.astype(np.float64), c["src"], nt)
    assert rel_l2(qa.double().cpu().numpy(), oqa) <= 1e-4
    assert rel_l2(g.domain(l0).double().cpu().numpy(), og.interior(lam0)) <= 1e-4
    assert rel_l2(g.domain(l1).double().cpu().numpy(), og.interior(lam1)) <= 1e-4
    g.close()
