"""GPU isotropic elastic propagation (velocity-stress, staggered grid)
against the FP64 oracle: every component and the traces on small grids with
damping, sources and receivers, zero and loopback halos, radius 1 to 8; the
benchmark's full 512^3 launch on sampled points; and the error paths."""
import numpy as np
import pytest

import oracle as O
import oracle.elastic as E
from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, to_dev, wrapped_boxes as _wrapped_boxes
import window_oracle as WO

pytestmark = pytest.mark.gpu


def _fd():
    from paper_2312_13094_amd import fd
    return fd


def _medium(shape, rng):
    vp = synth.minmax(synth.smooth_noise(shape, 2.5, rng), 2000.0, 3500.0).astype(np.float32)
    vs = (vp * synth.minmax(synth.smooth_noise(shape, 2.5, rng), 0.35, 0.6)).astype(np.float32)
    rho = synth.minmax(synth.smooth_noise(shape, 2.5, rng), 1600.0, 2600.0).astype(np.float32)
    return vp, vs, rho


def _gpu_run(shape, h, so, dt, nbl, bc, vp, vs, rho, src, q, rec, nt, state=None, tile=None):
    import torch
    FD = _fd()
    g = FD.Grid(shape, h, so, dt, 3500.0, nbl=nbl, boundary=bc, physics=FD.FD_ELASTIC)
    if tile is not None:
        g.set_tile(*tile)
    g.set_model(to_dev(vp), [to_dev(vs), to_dev(rho)])
    f = [g.field() for _ in range(9)]
    if state is not None:
        for k, name in enumerate(FD.ELASTIC_FIELDS):
            g.domain(f[k]).copy_(to_dev(state[name]))
    S = g.sparse(src) if src is not None else None
    R = g.sparse(rec) if rec is not None else None
    d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda") if R is not None else None
    g.forward(f, S, None if q is None else to_dev(q), R, d, nt)
    torch.cuda.synchronize()
    out = {name: g.domain(f[k]).double().cpu().numpy() for k, name in enumerate(FD.ELASTIC_FIELDS)}
    dd = None if d is None else d.double().cpu().numpy()
    g.close()
    return out, dd


@pytest.mark.parametrize("tile", [None, (0,)], ids=["zmarch", "points"])
@pytest.mark.parametrize("shape,so,nbl,bc", [
    ((20, 22, 70), 8, 4, 0),      # two 64-column tiles with a ragged tail, sponge
    ((17, 13, 19), 4, 3, 1),      # loopback halos of all nine components
    ((16, 18, 21), 16, 0, 1),     # radius 8
    ((9, 10, 11), 2, 2, 0),       # radius 1
    ((24, 20, 66), 8, 5, 1),
])
def test_elastic_matches_oracle(shape, so, nbl, bc, tile):
    rng = np.random.default_rng(sum(shape) + so)
    h = (10.0, 9.0, 11.0)
    vp, vs, rho = _medium(shape, rng)
    dt = synth.elastic_stable_dt(so, min(h), 3500.0)
    nt = 30
    src = np.array([[(s - 1) * hh * f for s, hh, f in zip(shape, h, (0.41, 0.52, 0.37))]])
    rec = np.stack([rng.uniform(0.0, (s - 1) * hh, 16) for s, hh in zip(shape, h)], 1)
    q = (synth.ricker(nt, dt, 60.0, t0=0.01)[:, None] * 1e6).astype(np.float32)
    # a non-zero start in every component (at n - 1/2 and n), so every
    # coupling term and every halo is exercised from the first update
    state = {f: (rng.standard_normal(shape) * (1e-3 if f[0] == "v" else 1e3)).astype(np.float32)
             for f in E.FIELDS}
    got, dg = _gpu_run(shape, h, so, dt, nbl, bc, vp, vs, rho, src, q, rec, nt, state, tile)
    og = O.Grid(shape, h, so=so, dt=dt, nbl=nbl, vmax=3500.0, bc=bc)
    ost = E.zero_state(og)
    for f in E.FIELDS:
        og.interior(ost[f])[...] = state[f].astype(np.float64)
    want, dw = E.forward(og, vp.astype(np.float64), vs.astype(np.float64),
                         rho.astype(np.float64), src=src, q=q.astype(np.float64), rec=rec, nt=nt,
                         state=ost)
    for f in E.FIELDS:
        err = rel_l2(got[f], og.interior(want[f]))
        assert err <= 2e-5, (f, err)
    assert rel_l2(dg, dw) <= 2e-5


@pytest.mark.parametrize("so", [4, 8, 12])
def test_elastic_zmarch_bit_identical_across_chunks(so):
    """The z-marching passes give identical bits for every z chunk and both
    tile shapes (the arithmetic of a point does not depend on the tiling); the
    one-thread-per-point passes agree with them to FP32 rounding (the
    compiler may fuse their multiply-adds differently)."""
    rng = np.random.default_rng(so)
    shape, h = (21, 19, 70), (10.0, 9.0, 11.0)
    vp, vs, rho = _medium(shape, rng)
    dt = synth.elastic_stable_dt(so, min(h), 3500.0)
    nt = 12
    src = np.array([[80.0, 90.0, 300.0]])
    rec = np.stack([rng.uniform(0.0, (s - 1) * hh, 10) for s, hh in zip(shape, h)], 1)
    q = (synth.ricker(nt, dt, 60.0, t0=0.01)[:, None] * 1e6).astype(np.float32)
    state = {f: (rng.standard_normal(shape) * (1e-3 if f[0] == "v" else 1e3)).astype(np.float32)
             for f in E.FIELDS}
    base = None
    for tile in [(4, 2, 64, 0), (4, 2, 5, 0), (4, 2, 1, 0), (4, 2, 21, 0), (8, 1, 64, 0),
                 (8, 1, 7, 0), (8, 2, 64, 0), (8, 2, 3, 0)]:
        got, d = _gpu_run(shape, h, so, dt, 4, 1, vp, vs, rho, src, q, rec, nt, state, tile)
        if base is None:
            base = (got, d)
            continue
        for f in E.FIELDS:
            np.testing.assert_array_equal(got[f], base[0][f], err_msg=str((tile, f)))
        np.testing.assert_array_equal(d, base[1])
    got, d = _gpu_run(shape, h, so, dt, 4, 1, vp, vs, rho, src, q, rec, nt, state, (0,))
    for f in E.FIELDS:
        assert rel_l2(got[f], base[0][f]) <= 1e-6, f
    assert rel_l2(d, base[1]) <= 1e-6


def test_elastic_source_only_first_update():
    """From rest, one update: velocities zero, each normal stress holds
    dt q w / h^3 at the source's nodes; receivers read the stress trace."""
    import torch
    FD = _fd()
    shape, h, so = (12, 13, 14), (10.0, 10.0, 10.0), 8
    dt = synth.elastic_stable_dt(so, 10.0, 3500.0)
    vp = np.full(shape, 3000.0, np.float32)
    vs = np.full(shape, 1500.0, np.float32)
    rho = np.full(shape, 2000.0, np.float32)
    pos = np.array([[5.25 * h[0], 6.5 * h[1], 7.75 * h[2]]])
    got, d = _gpu_run(shape, h, so, dt, 0, 0, vp, vs, rho, pos, np.array([[2.5]], np.float32), pos, 1)
    og = O.Grid(shape, h, so=so, dt=dt)
    want, dw = E.forward(og, vp, vs, rho, src=pos, q=np.array([[2.5]]), rec=pos, nt=1)
    for f in ("txx", "tyy", "tzz"):
        np.testing.assert_allclose(got[f], og.interior(want[f]), rtol=1e-6, atol=0)
    for f in ("vx", "vy", "vz", "txy", "txz", "tyz"):
        assert not got[f].any()
    np.testing.assert_allclose(d, dw, rtol=1e-6)
    del torch


def test_elastic_full_size_sampled_points():
    """The benchmark's launch (512^3, so 8, layered medium, 40-point sponge,
    loopback halos) for one update from a random state, checked at 24
    sampled points: 8 deep inside, 8 inside the damping layer and 8 within 3r
    of a face.  Each sample's oracle runs the two half steps on the window of
    half-width 2r (plus an r-wide halo) around it, taken with the periodic
    halo's wrapped indices and carrying the whole grid's medium coefficients
    and damping rate."""
    import torch
    FD = _fd()
    c = synth.cfg_elastic(n=512, nt=1)
    r = c.so // 2
    g = FD.Grid(c.shape, c.spacing, c.so, c.dt, c.vmax, nbl=c.nbl, boundary=c.boundary,
                physics=FD.FD_ELASTIC)
    vp, vs, rho = (torch.from_numpy(p).cuda() for p in (c.vp_profile, c.vs_profile, c.rho_profile))
    n = c.shape[0]
    full = [t[:, None, None].expand(n, n, n).contiguous() for t in (vp, vs, rho)]
    g.set_model(full[0], full[1:])
    del full
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    f = [g.field() for _ in range(9)]
    for k, name in enumerate(FD.ELASTIC_FIELDS):
        scale = 1e-3 if name[0] == "v" else 1e3
        g.domain(f[k]).copy_(torch.randn(c.shape, generator=gen, device="cuda") * scale)
    pts = np.concatenate(WO.sample_points(n, c.nbl, r, np.random.default_rng(5), 8))
    boxes = [_wrapped_boxes(g, f, FD.ELASTIC_FIELDS, pt, 3 * r) for pt in pts]
    g.forward(f, None, None, None, None, 1)
    torch.cuda.synchronize()
    got = [{name: float(g.domain(f[k])[tuple(pt)]) for k, name in enumerate(FD.ELASTIC_FIELDS)}
           for pt in pts]
    g.close()
    big = O.Grid(c.shape, c.spacing, so=c.so, dt=c.dt, nbl=c.nbl, vmax=c.vmax, bc=1)
    cols = [p.astype(np.float64)[:, None, None] for p in (c.vp_profile, c.vs_profile, c.rho_profile)]
    coef = E.staggered_params(*E.medium(*cols))
    for pt, box, gv in zip(pts, boxes, got):
        want = WO.step_at(big, "elastic", coef, box, pt)
        for name in E.FIELDS:
            mag = np.abs(box[name]).max()
            assert abs(gv[name] - want[name]) <= 1e-5 * mag, (name, tuple(pt), gv[name], want[name])


def test_elastic_errors():
    import torch
    FD = _fd()
    h = (10.0,) * 3
    dt = synth.elastic_stable_dt(8, 10.0, 3500.0)

    def code(fn):
        with pytest.raises(FD.FdError) as e:
            fn()
        return e.value.code

    assert code(lambda: FD.Grid((20, 20), (10.0, 10.0), 8, dt, 3500.0,
                                physics=FD.FD_ELASTIC)) == FD.FD_EINVAL
    assert code(lambda: FD.Grid((20, 20, 20), h, 8, dt, 3500.0, boundary=FD.FD_BC_EXTERNAL,
                                physics=FD.FD_ELASTIC)) == FD.FD_ENOTSUP
    assert code(lambda: FD.Grid((20, 20, 20), h, 8, 2.05 * dt, 3500.0,
                                physics=FD.FD_ELASTIC)) == FD.FD_EUNSTABLE
    g = FD.Grid((20, 20, 20), h, 8, dt, 3500.0, physics=FD.FD_ELASTIC)
    shape = (20, 20, 20)
    vp = torch.full(shape, 3000.0, device="cuda")
    rho = torch.full(shape, 2000.0, device="cuda")
    f = [g.field() for _ in range(9)]
    assert code(lambda: g.forward(f, nt=1)) == FD.FD_EINVAL                  # no model yet
    assert code(lambda: g.set_model(vp, [torch.full(shape, 2700.0, device="cuda"), rho])) \
        == FD.FD_EUNSTABLE                                                  # 3 lambda + 2 mu <= 0
    assert code(lambda: g.set_model(vp, [torch.full(shape, 1500.0, device="cuda"),
                                         -rho])) == FD.FD_EUNSTABLE
    assert code(lambda: g.set_model(torch.full(shape, 3600.0, device="cuda"),
                                    [torch.full(shape, 1500.0, device="cuda"), rho])) \
        == FD.FD_EUNSTABLE                                                  # above vmax
    assert code(lambda: g.set_model(vp, None)) == FD.FD_EINVAL
    g.set_model(vp, [torch.full(shape, 1500.0, device="cuda"), rho])
    assert code(lambda: g.forward(f[:8] + [f[0]], nt=1)) == FD.FD_EINVAL       # aliasing
    assert code(lambda: g.forward(f, nt=2, ckpt=[g.field() for _ in range(18)],
                                  ckpt_every=1)) == FD.FD_ENOTSUP
    assert code(lambda: g.step(f[0], f[1])) == FD.FD_ENOTSUP
    assert code(lambda: g.adjoint(f[:2], nt=1)) == FD.FD_ENOTSUP
    g.forward(f, nt=0)
    g.close()
