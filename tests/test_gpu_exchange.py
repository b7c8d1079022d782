"""Full exchange mode (the paper's "full" computation/communication pattern:
the halo update overlapped with the CORE, then the REMAINDER): against the
FP64 oracle directly (periodic halo, damping, sources and receivers), and
against basic mode bit for bit."""
import numpy as np
import pytest

from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, run_oracle_forward, to_dev

pytestmark = pytest.mark.gpu


def _fd():
    from paper_2312_13094_amd import fd
    return fd


def _case(shape, so, seed, nt):
    rng = np.random.default_rng(seed)
    h, vmax = 10.0, 3000.0
    v = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    src = np.array([[(s - 1) * h * f for s, f in zip(shape, (0.37, 0.61, 0.29))]])
    rec = np.stack([rng.uniform(0.0, (s - 1) * h, 20) for s in shape], 1)
    q = (synth.ricker(nt, dt, 25.0)[:, None] * 1e2).astype(np.float32)
    # a state that is non-zero at every face, so the exchanged halo matters
    u0 = rng.standard_normal(shape).astype(np.float32)
    um = rng.standard_normal(shape).astype(np.float32)
    return dict(h=h, vmax=vmax, v=v, dt=dt, src=src, rec=rec, q=q, u0=u0, um=um)


def _forward(shape, so, c, nt, nbl, tile, full):
    import torch
    FD = _fd()
    g = FD.Grid(shape, (c["h"],) * 3, so, c["dt"], c["vmax"], nbl=nbl,
                boundary=FD.FD_BC_LOOPBACK)
    if tile is not None:
        g.set_tile(*tile)
    if full:
        g.set_exchange_mode(FD.FD_XCHG_FULL)
    g.set_model(to_dev(c["v"]))
    a, b = g.field(), g.field()
    g.domain(a).copy_(to_dev(c["u0"]))
    g.domain(b).copy_(to_dev(c["um"]))
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda")
    g.forward([a, b], S, to_dev(c["q"]), R, d, nt)
    torch.cuda.synchronize()
    out = [g.domain(a).cpu().numpy(), g.domain(b).cpu().numpy(), d.cpu().numpy()]
    g.close()
    return out


@pytest.mark.parametrize("shape,so,tile", [
    ((24, 21, 70), 8, None),              # CORE x range crosses the first 64-column tile
    ((45, 38, 97), 8, (4, 4, 64, 1)),
    ((45, 38, 97), 8, (8, 2, 9, 7)),
    ((45, 38, 97), 8, (4, 1, 5, 4)),
    ((45, 38, 97), 8, (8, 2, 64, 28)),    # 128-wide tiles
    ((45, 38, 97), 8, (4, 2, 13, 29)),
    ((20, 19, 18), 16, None),             # radius 8: CORE 4 x 3 x 2
    ((9, 10, 130), 4, None),
    ((3, 4, 5), 2, (4, 1, 1, 0)),         # radius 1, single-point-deep CORE
    ((64, 80, 200), 8, None),
])
def test_full_mode_matches_basic(shape, so, tile):
    nt, nbl = 7, (3 if min(shape) > 8 else 0)
    c = _case(shape, so, 31, nt)
    basic = _forward(shape, so, c, nt, nbl, tile, False)
    full = _forward(shape, so, c, nt, nbl, tile, True)
    for x, y in zip(full, basic):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("shape,so,tile,nt", [
    ((24, 21, 70), 8, None, 1),
    ((45, 38, 97), 8, (8, 2, 64, 28), 1),
    ((20, 19, 18), 16, None, 1),
    ((45, 38, 97), 8, None, 40),
    ((45, 38, 97), 4, (4, 2, 13, 29), 40),
    ((64, 80, 200), 8, None, 40),
])
def test_full_mode_matches_oracle(shape, so, tile, nt):
    """Full mode against the FP64 oracle with periodic (loopback) halos, a
    damping layer, an off-grid source and 20 receivers, from a state that is
    non-zero at every face: fields and traces within 1e-5 after one step and
    1e-4 after 40."""
    nbl = 3 if min(shape) > 8 else 0
    c = _case(shape, so, 37, nt)
    full = _forward(shape, so, c, nt, nbl, tile, True)
    ou, oum, od = run_oracle_forward(shape, (c["h"],) * 3, so, c["dt"], c["vmax"], c["v"], nt,
                                     nbl=nbl, boundary=1, src=c["src"], q=c["q"], rec=c["rec"],
                                     u0=c["u0"], um=c["um"])
    tol = 1e-5 if nt == 1 else 1e-4
    assert rel_l2(full[0], ou) <= tol
    assert rel_l2(full[1], oum) <= tol
    assert rel_l2(full[2], od) <= tol


def test_full_mode_layered_workload_matches_oracle():
    """The headline recipe at 96^3 (layered velocity, 16-point sponge, Ricker,
    receiver line, loopback exchange every step), 300 steps in full mode:
    within 1e-4 of the oracle."""
    import torch
    FD = _fd()
    c = synth.cfg_3d_layered(n=96, nt=300, nbl=16)
    g = FD.Grid(c.shape, c.spacing, c.so, c.dt, c.vmax, nbl=c.nbl, boundary=FD.FD_BC_LOOPBACK)
    g.set_exchange_mode(FD.FD_XCHG_FULL)
    g.set_model(to_dev(c.velocity()))
    a, b = g.field(), g.field()
    S, R = g.sparse(c.src), g.sparse(c.rec)
    d = torch.zeros((c.nt, R.n), dtype=torch.float32, device="cuda")
    g.forward([a, b], S, to_dev(c.q), R, d, c.nt)
    torch.cuda.synchronize()
    gu, gd = g.domain(a).double().cpu().numpy(), d.double().cpu().numpy()
    g.close()
    ou, _, od = run_oracle_forward(c.shape, c.spacing, c.so, c.dt, c.vmax, c.velocity(), c.nt,
                                   nbl=c.nbl, boundary=c.boundary, src=c.src, q=c.q, rec=c.rec)
    assert rel_l2(gu, ou) <= 1e-4
    assert rel_l2(gd, od) <= 1e-4
    assert np.abs(od).max() > 0


def test_full_mode_step_loop_and_switch_back():
    """fd_step in full mode equals fd_forward in basic mode; switching back to
    basic mode on the same handle gives the basic result again."""
    import torch
    FD = _fd()
    shape, so, nt = (30, 26, 75), 8, 6
    c = _case(shape, so, 5, nt)
    ref = _forward(shape, so, c, nt, 4, None, False)
    g = FD.Grid(shape, (c["h"],) * 3, so, c["dt"], c["vmax"], nbl=4, boundary=FD.FD_BC_LOOPBACK)
    g.set_model(to_dev(c["v"]))
    S, R = g.sparse(c["src"]), g.sparse(c["rec"])
    qd = to_dev(c["q"])
    for mode in (FD.FD_XCHG_FULL, FD.FD_XCHG_BASIC):
        g.set_exchange_mode(mode)
        cur, prev = g.field(), g.field()
        g.domain(cur).copy_(to_dev(c["u0"]))
        g.domain(prev).copy_(to_dev(c["um"]))
        d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda")
        for n in range(nt):
            g.step(cur, prev, S, qd[n], R, d[n])
            cur, prev = prev, cur
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.domain(cur).cpu().numpy(), ref[0])
        np.testing.assert_array_equal(g.domain(prev).cpu().numpy(), ref[1])
        np.testing.assert_array_equal(d.cpu().numpy(), ref[2])
    g.close()


def test_full_mode_gradient_matches_basic():
    """The checkpointed imaging gradient (forward, recomputation and adjoint
    all in full mode) equals basic mode's bit for bit."""
    import torch
    FD = _fd()
    shape, so, nt, k = (26, 30, 70), 8, 23, 6
    c = _case(shape, so, 17, nt)
    grads = []
    for full in (False, True):
        g = FD.Grid(shape, (c["h"],) * 3, so, c["dt"], c["vmax"], nbl=5,
                    boundary=FD.FD_BC_LOOPBACK)
        if full:
            g.set_exchange_mode(FD.FD_XCHG_FULL)
        g.set_model(to_dev(c["v"]))
        S, R = g.sparse(c["src"]), g.sparse(c["rec"])
        q = to_dev(c["q"])
        nck = (nt + k - 1) // k
        ckpt = [g.field() for _ in range(2 * nck)]
        a, b = g.field(), g.field()
        d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda")
        g.forward([a, b], S, q, R, d, nt, ckpt=ckpt, ckpt_every=k)
        resid = to_dev(np.random.default_rng(4).standard_normal((nt, R.n)).astype(np.float32))
        la, lb = g.field(), g.field()
        qa = torch.zeros((nt, S.n), dtype=torch.float32, device="cuda")
        gm = torch.zeros(shape, dtype=torch.float32, device="cuda")
        slots = [g.field() for _ in range(k + 2)]
        g.adjoint([la, lb], R, resid, S, q, qa, nt, ckpt=ckpt, ckpt_every=k, slots=slots,
                  grad_m=gm)
        torch.cuda.synchronize()
        grads.append((d.cpu().numpy(), gm.cpu().numpy()))
        g.close()
    assert np.abs(grads[0][1]).max() > 0
    np.testing.assert_array_equal(grads[1][0], grads[0][0])
    np.testing.assert_array_equal(grads[1][1], grads[0][1])


def test_full_mode_rejections():
    FD = _fd()
    h, vmax = 10.0, 3000.0
    dt = synth.stable_dt(8, 3, h, vmax)

    def code(fn):
        with pytest.raises(FD.FdError) as e:
            fn()
        return e.value.code

    g = FD.Grid((20, 20, 40), (h,) * 3, 8, dt, vmax)          # zero boundary: nothing to overlap
    assert code(lambda: g.set_exchange_mode(FD.FD_XCHG_FULL)) == FD.FD_ENOTSUP
    g.close()
    g = FD.Grid((8, 20, 40), (h,) * 3, 8, dt, vmax, boundary=FD.FD_BC_LOOPBACK)   # nz <= 2r
    assert code(lambda: g.set_exchange_mode(FD.FD_XCHG_FULL)) == FD.FD_ENOTSUP
    g.close()
    dt2 = synth.stable_dt(8, 2, h, vmax)
    g = FD.Grid((40, 40), (h,) * 2, 8, dt2, vmax, boundary=FD.FD_BC_LOOPBACK)     # 2-D
    assert code(lambda: g.set_exchange_mode(FD.FD_XCHG_FULL)) == FD.FD_ENOTSUP
    g.close()
    g = FD.Grid((20, 20, 40), (h,) * 3, 8, dt, vmax, boundary=FD.FD_BC_LOOPBACK)
    assert code(lambda: g.set_exchange_mode(7)) == FD.FD_EINVAL
    g.set_tile(0)
    assert code(lambda: g.set_exchange_mode(FD.FD_XCHG_FULL)) == FD.FD_ENOTSUP
    g.set_tile(4, 4, 16, 12)
    g.set_exchange_mode(FD.FD_XCHG_FULL)
    assert code(lambda: g.set_tile(0)) == FD.FD_EINVAL
    g.set_exchange_mode(FD.FD_XCHG_BASIC)
    g.set_tile(0)
    g.close()
