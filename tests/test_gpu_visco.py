"""GPU visco-elastic propagation (one relaxation mechanism) against the FP64
oracle: all fifteen components and the traces on small grids (damping,
sources, receivers, zero and loopback halos, radius 1 to 8, both velocity
kernels), the benchmark's 512^3 launch on sampled points, and the error
paths."""
import numpy as np
import pytest

import oracle as O
import oracle.visco as V
from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, to_dev, wrapped_boxes as _wrapped_boxes
import window_oracle as WO

pytestmark = pytest.mark.gpu


def _fd():
    from paper_2312_13094_amd import fd
    return fd


def _medium(shape, rng):
    vp = synth.minmax(synth.smooth_noise(shape, 2.5, rng), 2000.0, 3200.0)
    vs = vp * synth.minmax(synth.smooth_noise(shape, 2.5, rng), 0.4, 0.6)
    rho = synth.minmax(synth.smooth_noise(shape, 2.5, rng), 1600.0, 2600.0)
    qp = synth.minmax(synth.smooth_noise(shape, 2.5, rng), 8.0, 40.0)
    tep, ts = synth.sls_times(qp, 25.0)
    tes = ts * synth.minmax(synth.smooth_noise(shape, 2.5, rng), 1.05, 1.4)
    return [a.astype(np.float32) for a in (vp, vs, rho, tep, tes, ts)]


def _gpu_run(shape, h, so, dt, vmax, nbl, bc, med, src, q, rec, nt, state=None, tile=None):
    import torch
    FD = _fd()
    g = FD.Grid(shape, h, so, dt, vmax, nbl=nbl, boundary=bc, physics=FD.FD_VISCO)
    if tile is not None:
        g.set_tile(*tile)
    g.set_model(to_dev(med[0]), [to_dev(a) for a in med[1:]])
    f = [g.field() for _ in range(15)]
    if state is not None:
        for k, name in enumerate(FD.VISCO_FIELDS):
            g.domain(f[k]).copy_(to_dev(state[name]))
    S = g.sparse(src) if src is not None else None
    R = g.sparse(rec) if rec is not None else None
    d = torch.zeros((nt, R.n), dtype=torch.float32, device="cuda") if R is not None else None
    g.forward(f, S, None if q is None else to_dev(q), R, d, nt)
    torch.cuda.synchronize()
    out = {name: g.domain(f[k]).double().cpu().numpy() for k, name in enumerate(FD.VISCO_FIELDS)}
    dd = None if d is None else d.double().cpu().numpy()
    g.close()
    return out, dd


@pytest.mark.parametrize("tile", [None, (0,)], ids=["zmarch", "points"])
@pytest.mark.parametrize("shape,so,nbl,bc", [
    ((20, 22, 70), 8, 4, 0),
    ((17, 13, 19), 4, 3, 1),
    ((16, 18, 21), 16, 0, 1),
    ((9, 10, 11), 2, 2, 0),
])
def test_visco_matches_oracle(shape, so, nbl, bc, tile):
    rng = np.random.default_rng(sum(shape) + 3 * so)
    h = (10.0, 9.0, 11.0)
    med = _medium(shape, rng)
    vmax = float((med[0] * np.sqrt(med[3] / med[5])).max()) * 1.001
    dt = synth.elastic_stable_dt(so, min(h), vmax)
    nt = 30
    src = np.array([[(s - 1) * hh * f for s, hh, f in zip(shape, h, (0.41, 0.52, 0.37))]])
    rec = np.stack([rng.uniform(0.0, (s - 1) * hh, 16) for s, hh in zip(shape, h)], 1)
    q = (synth.ricker(nt, dt, 60.0, t0=0.01)[:, None] * 1e6).astype(np.float32)
    state = {f: (rng.standard_normal(shape) * (1e-3 if f[0] == "v" else 1e3)).astype(np.float32)
             for f in V.FIELDS}
    got, dg = _gpu_run(shape, h, so, dt, vmax, nbl, bc, med, src, q, rec, nt, state, tile)
    og = O.Grid(shape, h, so=so, dt=dt, nbl=nbl, vmax=vmax, bc=bc)
    ost = V.zero_state(og)
    for f in V.FIELDS:
        og.interior(ost[f])[...] = state[f].astype(np.float64)
    want, dw = V.forward(og, *[a.astype(np.float64) for a in med], src=src,
                         q=q.astype(np.float64), rec=rec, nt=nt, state=ost)
    for f in V.FIELDS:
        err = rel_l2(got[f], og.interior(want[f]))
        assert err <= 2e-5, (f, err)
    assert rel_l2(dg, dw) <= 2e-5


def test_visco_full_size_sampled_points():
    """The benchmark's launch (512^3, so 8, layered medium with Qp = 40 vp /
    1 km/s, Qs = Qp / 2, 40-point sponge, loopback halos) for one update from
    a random state, checked at 18 sampled points (6 deep inside, 6 inside the
    damping layer, 6 within 3r of a face) against the oracle's two half steps
    on the wrapped window around each, with the whole grid's coefficients and
    damping rate."""
    import torch
    FD = _fd()
    c = synth.cfg_visco(n=512, nt=1)
    r = c.so // 2
    g = FD.Grid(c.shape, c.spacing, c.so, c.dt, c.vmax, nbl=c.nbl, boundary=c.boundary,
                physics=FD.FD_VISCO)
    n = c.shape[0]
    prof = [torch.from_numpy(p).cuda()[:, None, None].expand(n, n, n).contiguous()
            for p in c.profiles()]
    g.set_model(prof[0], prof[1:])
    del prof
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    f = [g.field() for _ in range(15)]
    for k, name in enumerate(FD.VISCO_FIELDS):
        scale = 1e-3 if name[0] == "v" else 1e3
        g.domain(f[k]).copy_(torch.randn(c.shape, generator=gen, device="cuda") * scale)
    pts = np.concatenate(WO.sample_points(n, c.nbl, r, np.random.default_rng(6), 6))
    boxes = [_wrapped_boxes(g, f, FD.VISCO_FIELDS, pt, 3 * r) for pt in pts]
    g.forward(f, None, None, None, None, 1)
    torch.cuda.synchronize()
    got = [{name: float(g.domain(f[k])[tuple(pt)]) for k, name in enumerate(FD.VISCO_FIELDS)}
           for pt in pts]
    g.close()
    big = O.Grid(c.shape, c.spacing, so=c.so, dt=c.dt, nbl=c.nbl, vmax=c.vmax, bc=1)
    coef = V.coefficients(*(p.astype(np.float64)[:, None, None] for p in c.profiles()))
    for pt, box, gv in zip(pts, boxes, got):
        want = WO.step_at(big, "visco", coef, box, pt)
        for name in V.FIELDS:
            mag = np.abs(box[name]).max()
            assert abs(gv[name] - want[name]) <= 1e-5 * mag, (name, tuple(pt), gv[name], want[name])


def test_visco_errors():
    import torch
    FD = _fd()
    h = (10.0,) * 3
    dt = synth.elastic_stable_dt(8, 10.0, 3500.0)

    def code(fn):
        with pytest.raises(FD.FdError) as e:
            fn()
        return e.value.code

    assert code(lambda: FD.Grid((20, 20), (10.0, 10.0), 8, dt, 3500.0,
                                physics=FD.FD_VISCO)) == FD.FD_EINVAL
    assert code(lambda: FD.Grid((20, 20, 20), h, 8, dt, 3500.0, boundary=FD.FD_BC_EXTERNAL,
                                physics=FD.FD_VISCO)) == FD.FD_ENOTSUP
    shape = (20, 20, 20)
    g = FD.Grid(shape, h, 8, dt, 3500.0, physics=FD.FD_VISCO)
    full = lambda v: torch.full(shape, v, device="cuda")
    ok = [full(1500.0), full(2000.0), full(0.012), full(0.011), full(0.01)]
    f = [g.field() for _ in range(15)]
    assert code(lambda: g.forward(f, nt=1)) == FD.FD_EINVAL                  # no model yet
    assert code(lambda: g.set_model(full(3000.0), ok[:4])) == FD.FD_EINVAL      # four aux only
    bad_ts = ok[:4] + [full(0.5 * dt)]                                          # tau_s < dt
    assert code(lambda: g.set_model(full(3000.0), bad_ts)) == FD.FD_EUNSTABLE
    bad_te = [ok[0], ok[1], full(0.009), ok[3], ok[4]]                          # tau_ep < tau_s
    assert code(lambda: g.set_model(full(3000.0), bad_te)) == FD.FD_EUNSTABLE
    big = [ok[0], ok[1], full(0.02), ok[3], ok[4]]                              # unrelaxed vp > vmax
    assert code(lambda: g.set_model(full(3000.0), big)) == FD.FD_EUNSTABLE
    g.set_model(full(3000.0), ok)
    assert code(lambda: g.forward(f[:14] + [f[3]], nt=1)) == FD.FD_EINVAL      # aliasing
    assert code(lambda: g.set_tile(8, 4, 64, 0)) == FD.FD_EINVAL
    assert code(lambda: g.adjoint(f[:2], nt=1)) == FD.FD_ENOTSUP
    g.forward(f, nt=0)
    g.close()
