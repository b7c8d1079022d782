"""GPU parity of the acoustic hot path (HIP kernels via the C ABI) against
the FP64 oracle on the same seeded inputs.

Tolerances: relative L2 <= 1e-5 after one step, <= 1e-4 after a full run
(fields and traces); integer/byte work (halo pack/unpack, subdomain
emulation, tile independence) is bit-exact.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, run_gpu_forward, run_oracle_forward, to_dev

pytestmark = pytest.mark.gpu


def _fd():
    from paper_2312_13094_amd import fd
    return fd


def _sparse_points(shape, h, n, rng, margin=0):
    return np.stack([rng.uniform(margin * h, (s - 1 - margin) * h, n) for s in shape], 1)


# ---------------------------------------------------------------------------
# halo faces: bit-exact against the oracle's pack/unpack
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,so", [((21, 19, 70), 8), ((9, 33, 65), 4), ((40, 37), 12),
                                      ((17, 16, 130), 16)])
def test_pack_unpack_bit_exact(shape, so):
    import torch
    FD = _fd()
    rng = np.random.default_rng(0)
    g = FD.Grid(shape, (10.0,) * len(shape), so, 1e-4, 1000.0)
    og = O.Grid(shape, (10.0,) * len(shape), so=so, dt=1e-4)
    f = g.field()
    f.copy_(torch.from_numpy(rng.standard_normal(g.field_elems).astype(np.float32)))
    bufs = [torch.full((max(g.face_elems(k), 1),), float("nan"), device="cuda") for k in range(6)]
    g.pack_halo(f, bufs)
    torch.cuda.synchronize()
    ref = og.zeros()
    r = so // 2
    ref[...] = g.with_halo(f).double().cpu().numpy()
    for k in range(6):
        n = og_face = O.face_elems(og, k)
        assert g.face_elems(k) == og_face
        if n:
            np.testing.assert_array_equal(bufs[k][:n].double().cpu().numpy(), O.pack_face(og, ref, k))
    # unpack fresh random buffers into every halo face
    new = [torch.from_numpy(rng.standard_normal(max(g.face_elems(k), 1)).astype(np.float32)).cuda()
           for k in range(6)]
    g.unpack_halo(f, new)
    torch.cuda.synchronize()
    for k in range(6):
        n = O.face_elems(og, k)
        if n:
            O.unpack_face(og, ref, k, new[k][:n].double().cpu().numpy())
    np.testing.assert_array_equal(g.with_halo(f).double().cpu().numpy(), ref)
    del r


@pytest.mark.parametrize("shape,so", [((12, 10, 40), 8), ((9, 11, 13), 6), ((14, 37), 4),
                                      ((12, 10, 64), 8), ((10, 9, 32), 16), ((8, 7, 96), 8)])
def test_loopback_exchange_equals_pack_then_unpack(shape, so):
    """The fused loopback exchange inside a loopback update leaves the
    current field exactly as the oracle's face pack followed by unpack of
    the opposite face's buffer (periodic self-neighbour) would."""
    import torch
    FD = _fd()
    rng = np.random.default_rng(5)
    h = (10.0,) * len(shape)
    dt = 1e-4                     # far inside the stability limit of every order
    g = FD.Grid(shape, h, so, dt, 3000.0, boundary=FD.FD_BC_LOOPBACK)
    g.set_model(to_dev(np.full(shape, 2000.0, np.float32)))
    og = O.Grid(shape, h, so=so, dt=dt)
    a, b = g.field(), g.field()
    a.copy_(torch.from_numpy(rng.standard_normal(g.field_elems).astype(np.float32)))
    ref = og.zeros()
    ref[...] = g.with_halo(a).double().cpu().numpy()
    packed = [O.pack_face(og, ref, k) if O.face_elems(og, k) else None for k in range(6)]
    for k in range(6):
        if packed[k ^ 1] is not None:
            O.unpack_face(og, ref, k, packed[k ^ 1])
    g.step(a, b)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g.with_halo(a).double().cpu().numpy(), ref)


def test_pack_rejects_bad_face_mask():
    import torch
    FD = _fd()
    g = FD.Grid((8, 8, 8), (10.0,) * 3, 4, 1e-4, 1000.0)
    f = g.field()
    bufs = [torch.zeros(g.face_elems(k), device="cuda") for k in range(6)]
    with pytest.raises(FD.FdError):
        g.pack_halo(f, bufs, mask=0x40)
    bufs[3] = None
    with pytest.raises(FD.FdError):
        g.pack_halo(f, bufs)


# ---------------------------------------------------------------------------
# one step from a smooth random state
# ---------------------------------------------------------------------------

ONE_STEP = [
    # shape, so, nbl, boundary, tile
    ((37, 29, 101), 8, 6, 0, (4, 4, 16, 1)),
    ((37, 29, 101), 8, 6, 1, (4, 2, 64, 1)),
    ((33, 40, 70), 4, 5, 0, (8, 2, 8, 0)),
    ((26, 35, 66), 12, 4, 1, (4, 8, 64, 1)),
    ((34, 31, 65), 16, 8, 0, (2, 8, 16, 1)),
    ((30, 24, 64), 2, 3, 0, (4, 1, 7, 1)),
    ((22, 20, 90), 8, 4, 0, (0, 0, 0, 0)),     # one-thread-per-point kernel
    ((168, 168), 4, 20, 0, None),
    ((50, 77), 8, 10, 1, None),
]


@pytest.mark.parametrize("shape,so,nbl,bc,tile", ONE_STEP)
def test_one_step_parity(shape, so, nbl, bc, tile):
    rng = np.random.default_rng(10 + so)
    ndim = len(shape)
    h = 10.0
    vmax = 4000.0
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, ndim, h, vmax)
    u0 = synth.smooth_state(shape, 1, 4.0)
    um = (0.9 * u0 + 0.1 * synth.smooth_state(shape, 2, 4.0)).astype(np.float32)
    src = _sparse_points(shape, h, 3, rng)
    rec = _sparse_points(shape, h, 40, rng)
    q = rng.standard_normal((1, 3)).astype(np.float32) * 1e3
    args = dict(shape=shape, spacing=(h,) * ndim, so=so, dt=dt, vmax=vmax, v=v, nt=1, nbl=nbl,
                boundary=bc, src=src, q=q, rec=rec, u0=u0, um=um)
    gu, gum, gd = run_gpu_forward(tile=tile, **args)
    ou, oum, od = run_oracle_forward(**args)
    assert rel_l2(gu, ou) <= 1e-5
    np.testing.assert_array_equal(gum, u0.astype(np.float64))   # u^0 handed back unchanged
    assert rel_l2(gd, od) <= 1e-5


def test_tiles_are_bit_identical():
    """The per-point arithmetic does not depend on the tile, the z chunk, the
    XCD remap, the prefetch distance, the halo-ring loads or the cache hints."""
    rng = np.random.default_rng(3)
    shape, so, h, vmax = (45, 38, 97), 8, 10.0, 3000.0
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    u0 = synth.smooth_state(shape, 5, 3.0)
    base = None
    for tile in [(4, 4, 64, 1), (4, 1, 5, 0), (4, 2, 13, 1), (4, 8, 45, 1), (8, 2, 9, 1),
                 (8, 4, 64, 0), (2, 8, 3, 1), (4, 4, 64, 2), (4, 4, 7, 3), (4, 2, 13, 6),
                 (8, 2, 9, 7), (4, 1, 5, 4), (4, 4, 64, 8), (8, 4, 11, 12), (4, 2, 3, 13),
                 (2, 8, 64, 9), (8, 2, 64, 12), (8, 4, 128, 12), (8, 2, 64, 28),
                 (4, 4, 7, 20), (4, 4, 11, 16), (4, 2, 13, 29), (8, 2, 64, 30),
                 (8, 2, 9, 31), (4, 4, 11, 26), (4, 1, 5, 10), (8, 4, 7, 14)]:
        u, _, _ = run_gpu_forward(shape, (h,) * 3, so, dt, vmax, v, 5, nbl=7, u0=u0, tile=tile)
        if base is None:
            base = u
        else:
            np.testing.assert_array_equal(u, base)


# ---------------------------------------------------------------------------
# full runs
# ---------------------------------------------------------------------------

def test_2d_homogeneous_full_run():
    """168 x 168 (128^2 + 20-point sponge), so 4, 200 steps, Ricker at the
    centre, 128 receivers: fields and traces within 1e-4 of the oracle."""
    c = synth.cfg_2d()
    args = dict(shape=c.shape, spacing=c.spacing, so=c.so, dt=c.dt, vmax=c.vmax,
                v=c.velocity(), nt=c.nt, nbl=c.nbl, boundary=c.boundary, src=c.src, q=c.q,
                rec=c.rec)
    gu, gum, gd = run_gpu_forward(**args)
    ou, oum, od = run_oracle_forward(**args)
    assert rel_l2(gu, ou) <= 1e-4
    assert rel_l2(gum, oum) <= 1e-4
    assert rel_l2(gd, od) <= 1e-4
    assert np.abs(od).max() > 0


@pytest.mark.parametrize("tile", [None, (4, 2, 32, 1)])
def test_3d_layered_loopback_full_run(tile):
    """The layered so-8 workload at 96^3 (same recipe as the 512^3 headline:
    sponge, Ricker, receiver line, loopback halo exchange every step)."""
    c = synth.cfg_3d_layered(n=96, nt=300, nbl=16)
    args = dict(shape=c.shape, spacing=c.spacing, so=c.so, dt=c.dt, vmax=c.vmax,
                v=c.velocity(), nt=c.nt, nbl=c.nbl, boundary=c.boundary, src=c.src, q=c.q,
                rec=c.rec)
    gu, _, gd = run_gpu_forward(tile=tile, **args)
    ou, _, od = run_oracle_forward(**args)
    assert rel_l2(gu, ou) <= 1e-4
    assert rel_l2(gd, od) <= 1e-4


def test_nan_in_padding_never_reaches_domain():
    """Poison everything outside DOMAIN + halo (x padding) and the halo edges
    and corners: a star stencil must read none of it."""
    import torch
    FD = _fd()
    rng = np.random.default_rng(4)
    shape, so, h, vmax = (30, 27, 75), 8, 10.0, 3000.0
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    u0 = synth.smooth_state(shape, 6, 3.0)
    ref, _, _ = run_gpu_forward(shape, (h,) * 3, so, dt, vmax, v, 10, nbl=5, u0=u0)
    g = FD.Grid(shape, (h,) * 3, so, dt, vmax, nbl=5)
    g.set_model(to_dev(v))
    a, b = g.field(), g.field()
    for f in (a, b):
        f.fill_(float("nan"))
        hv = g.with_halo(f)
        r = so // 2
        hv[r:-r, r:-r, :] = 0.0     # halo faces along x zero
        hv[r:-r, :, r:-r] = 0.0     # halo faces along y zero
        hv[:, r:-r, r:-r] = 0.0     # halo faces along z zero
    g.domain(a).copy_(to_dev(u0))
    g.forward([a, b], nt=10)
    torch.cuda.synchronize()
    got = g.domain(a).double().cpu().numpy()
    assert np.isfinite(got).all()
    np.testing.assert_array_equal(got, ref)


# ---------------------------------------------------------------------------
# headline size (512^3, so 8): one step vs the oracle; 500 steps vs an exact
# discrete solution
# ---------------------------------------------------------------------------

def _plane_waves(shape, h, modes, phases):
    xs = [np.arange(n, dtype=np.float64) * h for n in shape]
    out = np.zeros(shape, dtype=np.float64)
    for m, ph in zip(modes, phases):
        k = [2 * math.pi * mi / (n * h) for mi, n in zip(m, shape)]
        out += np.cos(k[0] * xs[0][:, None, None] + k[1] * xs[1][None, :, None] +
                      k[2] * xs[2][None, None, :] + ph)
    return out


@pytest.mark.slow
def test_headline_512_one_step_vs_oracle():
    c = synth.cfg_3d_layered()
    u0 = _plane_waves(c.shape, 10.0, [(3, 5, 7), (11, 2, 6), (1, 13, 4)], [0.3, 1.1, 2.0])
    u0 = u0.astype(np.float32)
    um = (0.97 * u0).astype(np.float32)
    args = dict(shape=c.shape, spacing=c.spacing, so=c.so, dt=c.dt, vmax=c.vmax,
                v=c.velocity(), nt=1, nbl=c.nbl, boundary=c.boundary, src=c.src,
                q=(c.q[40:41] * 1e6).astype(np.float32), rec=c.rec, u0=u0, um=um)
    gu, _, gd = run_gpu_forward(**args)
    ou, _, od = run_oracle_forward(**args)
    assert rel_l2(gu, ou) <= 1e-5
    assert rel_l2(gd, od) <= 1e-5


@pytest.mark.slow
def test_headline_512_full_run_vs_oracle():
    """The headline workload exactly as bench.py times it: 512^3, so 8,
    layered velocity, 40-point sponge, 15 Hz Ricker, 512 receivers, loopback
    exchange of the six faces every step, 500 steps, default tile.  The final
    field, the previous field and all traces within 1e-4 relative L2 of the
    FP64 oracle (about 90 s of oracle time on 16 cores)."""
    c = synth.cfg_3d_layered()
    v = c.velocity()
    args = dict(shape=c.shape, spacing=c.spacing, so=c.so, dt=c.dt, vmax=c.vmax, v=v,
                nt=c.nt, nbl=c.nbl, boundary=c.boundary, src=c.src, q=c.q, rec=c.rec)
    gu, gum, gd = run_gpu_forward(**args)
    ou, oum, od = run_oracle_forward(**args)
    eu, eum, ed = rel_l2(gu, ou), rel_l2(gum, oum), rel_l2(gd, od)
    print("512^3 x 500 steps: field %.2e previous %.2e traces %.2e" % (eu, eum, ed))
    assert np.abs(od).max() > 0
    assert eu <= 1e-4 and eum <= 1e-4 and ed <= 1e-4


def _symbol(w, theta):
    return w[0] + 2 * sum(w[k] * math.cos(k * theta) for k in range(1, len(w)))


@pytest.mark.slow
def test_headline_512_plane_wave_500_steps():
    """512^3, so 8, loopback (periodic) halos every step, 500 steps: the
    discrete plane wave cos(k.x - w t) with sin^2(w dt/2) = -(v dt)^2/4 sum
    sigma(k_a h)/h^2 is exact; FP32 stays within 1e-4 relative L2.  The
    wavenumber sits in the workload's band (about 15 Hz at 3 km/s): FP32
    rounding in a leapfrog grows like sqrt(steps) eps / (w dt), so a far
    lower-frequency mode would measure that growth rather than the kernels."""
    import torch
    FD = _fd()
    n, so, h, v, nt = 512, 8, 10.0, 3000.0, 500
    dt = synth.stable_dt(so, 3, h, 4500.0)
    g = FD.Grid((n, n, n), (h,) * 3, so, dt, 4500.0, nbl=0, boundary=FD.FD_BC_LOOPBACK)
    g.set_model(torch.full((n, n, n), v, dtype=torch.float32, device="cuda"))
    w = O.d2_weights(so)  # FP64 weights, pinned by the oracle tests
    m = (15, 12, 17)
    k = [2 * math.pi * mi / (n * h) for mi in m]
    s2 = -(v * dt) ** 2 / 4 * sum(_symbol(w, kk * h) / h ** 2 for kk in k)
    om = 2 * math.asin(math.sqrt(s2)) / dt
    ph = (torch.arange(n, device="cuda", dtype=torch.float64) * h)
    phase = (k[0] * ph[:, None, None] + k[1] * ph[None, :, None] + k[2] * ph[None, None, :])
    a, b = g.field(), g.field()
    g.domain(a).copy_(torch.cos(phase).float())
    g.domain(b).copy_(torch.cos(phase + om * dt).float())
    g.forward([a, b], nt=nt)
    want = torch.cos(phase - om * nt * dt)
    got = g.domain(a).double()
    err = (torch.linalg.vector_norm(got - want) / torch.linalg.vector_norm(want)).item()
    assert err <= 1e-4, err


# ---------------------------------------------------------------------------
# multi-subdomain emulation on the device (external halos, pack/unpack)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("boundary", [0, 1])
def test_step_loop_equals_forward(boundary):
    """fd_step with alternating buffer roles reproduces fd_forward bit for
    bit: states, and traces sampled after every update."""
    import torch
    FD = _fd()
    rng = np.random.default_rng(12)
    shape, so, h, vmax, nt = (24, 21, 70), 8, 10.0, 3000.0, 9
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    src = np.array([[11.3 * h, 9.7 * h, 33.2 * h]])
    rec = np.array([[5 * h, 10.5 * h, (3 + 2 * i) * h] for i in range(30)])
    q = synth.ricker(nt, dt, 25.0)[:, None].astype(np.float32)
    u0 = synth.smooth_state(shape, 6, 3.0)
    g = FD.Grid(shape, (h,) * 3, so, dt, vmax, nbl=5, boundary=boundary)
    g.set_model(to_dev(v))
    S, R = g.sparse(src), g.sparse(rec)
    qd = to_dev(q)
    a, b = g.field(), g.field()
    g.domain(a).copy_(to_dev(u0))
    d_ref = torch.zeros((nt, R.n), device="cuda")
    g.forward([a, b], S, qd, R, d_ref, nt)
    c, e = g.field(), g.field()
    g.domain(c).copy_(to_dev(u0))
    d = torch.zeros_like(d_ref)
    cur, prev = c, e
    for n in range(nt):
        g.step(cur, prev, S, qd[n], R, d[n])
        cur, prev = prev, cur
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g.domain(cur).cpu().numpy(), g.domain(a).cpu().numpy())
    np.testing.assert_array_equal(g.domain(prev).cpu().numpy(), g.domain(b).cpu().numpy())
    np.testing.assert_array_equal(d.cpu().numpy(), d_ref.cpu().numpy())
    # fd_step_lagged: the same updates, each recording the level it reads
    # (update n records the result of update n - 1; the last level by
    # fd_sample)
    c2, e2 = g.field(), g.field()
    g.domain(c2).copy_(to_dev(u0))
    d2 = torch.zeros_like(d_ref)
    cur, prev = c2, e2
    for n in range(nt):
        g.step(cur, prev, S, qd[n], R if n else None, d2[n - 1] if n else None, lagged=True)
        cur, prev = prev, cur
    g.sample(cur, R, d2[nt - 1])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g.domain(cur).cpu().numpy(), g.domain(a).cpu().numpy())
    np.testing.assert_array_equal(d2.cpu().numpy(), d_ref.cpu().numpy())
    g.close()


XFACE_CASES = [
    # shape, so, source x positions (cells), tile (by, ry, nzb, flags)
    ((24, 21, 70), 8, [33.2, 1.5], (8, 2, 64, 28)),    # one 128-wide tile holds both x faces
    ((24, 21, 70), 8, [67.6], (4, 2, 13, 13)),         # within R of the x+ face; two 64-wide tiles
    ((24, 21, 70), 8, [0.0], (4, 4, 7, 8)),            # on the x- face itself
    ((20, 19, 40), 16, [20.3, 38.5], (4, 2, 9, 12)),   # radius 8
    ((24, 21, 70), 8, [68.9], (4, 2, 13, 5)),          # no halo-ring tile
    ((24, 21, 70), 8, [68.9], (0, 0, 0, 0)),           # one thread per point
    ((24, 21, 64), 8, [62.5, 30.1], (8, 2, 64, 28)),   # nx a multiple of 32: whole-line x faces
    ((20, 19, 64), 16, [0.5], (4, 2, 9, 12)),
]


@pytest.mark.parametrize("shape,so,sx,tile", XFACE_CASES)
def test_loopback_sources_next_to_x_faces(shape, so, sx, tile):
    """Loopback grid with sources injecting within R of the x faces (whose
    values the next exchange must carry into the opposite halo) and a
    receiver line across x: fd_forward equals a loop of fd_step bit for bit,
    fields and traces, and the oracle within 1e-5, over halo-ring tiles of
    one and two 64-wide columns per lane, other tiles and the
    one-thread-per-point kernel."""
    import torch
    FD = _fd()
    rng = np.random.default_rng(21)
    h, vmax, nt = 10.0, 3000.0, 9
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    src = np.array([[(shape[0] / 2 - 0.3) * h, (shape[1] / 2 + 0.2) * h, x * h] for x in sx])
    rec = np.array([[5 * h, 10.5 * h, (1 + 2 * i) * h] for i in range((shape[2] - 2) // 2)])
    q = (rng.standard_normal((nt, len(sx))) * 1e3).astype(np.float32)
    u0 = synth.smooth_state(shape, 6, 3.0)
    g = FD.Grid(shape, (h,) * 3, so, dt, vmax, nbl=5, boundary=1)
    g.set_tile(*tile)
    g.set_model(to_dev(v))
    S, R = g.sparse(src), g.sparse(rec)
    qd = to_dev(q)
    a, b = g.field(), g.field()
    g.domain(a).copy_(to_dev(u0))
    d_ref = torch.zeros((nt, R.n), device="cuda")
    g.forward([a, b], S, qd, R, d_ref, nt)
    c, e = g.field(), g.field()
    g.domain(c).copy_(to_dev(u0))
    d = torch.zeros_like(d_ref)
    cur, prev = c, e
    for n in range(nt):
        g.step(cur, prev, S, qd[n], R, d[n])
        cur, prev = prev, cur
    torch.cuda.synchronize()
    got = g.domain(a).cpu().numpy()
    np.testing.assert_array_equal(g.domain(cur).cpu().numpy(), got)
    np.testing.assert_array_equal(g.domain(prev).cpu().numpy(), g.domain(b).cpu().numpy())
    np.testing.assert_array_equal(d.cpu().numpy(), d_ref.cpu().numpy())
    dg = d_ref.cpu().numpy()
    g.close()
    ou, _, od = run_oracle_forward(shape, (h,) * 3, so, dt, vmax, v, nt, nbl=5, boundary=1,
                                   src=src, q=q, rec=rec, u0=u0)
    assert rel_l2(got, ou) <= 1e-5
    assert rel_l2(dg, od) <= 1e-5


def test_multidomain_emulation_bitwise():
    import torch
    FD = _fd()
    rng = np.random.default_rng(8)
    shape, so, h, vmax = (40, 36, 130), 8, 10.0, 3000.0
    split = (2, 2, 2)
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    u0 = synth.smooth_state(shape, 9, 3.0)
    nt = 8
    ref, _, _ = run_gpu_forward(shape, (h,) * 3, so, dt, vmax, v, nt, u0=u0)
    cuts = [np.array_split(np.arange(s), p) for s, p in zip(shape, split)]
    blocks = list(np.ndindex(*split))
    sub = {}
    for bk in blocks:
        sl = tuple(slice(c[i][0], c[i][-1] + 1) for c, i in zip(cuts, bk))
        g = FD.Grid(tuple(s.stop - s.start for s in sl), (h,) * 3, so, dt, vmax,
                    boundary=FD.FD_BC_EXTERNAL)
        g.set_model(to_dev(np.ascontiguousarray(v[sl])))
        a, b = g.field(), g.field()
        g.domain(a).copy_(to_dev(np.ascontiguousarray(u0[sl])))
        bufs = [torch.zeros(max(g.face_elems(k), 1), device="cuda") for k in range(6)]
        sub[bk] = dict(g=g, sl=sl, st=[a, b], bufs=bufs)
    for _ in range(nt):
        for bk in blocks:
            s = sub[bk]
            s["g"].pack_halo(s["st"][0], s["bufs"])
        for bk in blocks:
            s = sub[bk]
            recv = [None] * 6
            mask = 0
            for f in range(6):
                nb = list(bk)
                nb[f // 2] += 1 if f & 1 else -1
                if 0 <= nb[f // 2] < split[f // 2]:
                    recv[f] = sub[tuple(nb)]["bufs"][f ^ 1]
                    mask |= 1 << f
            s["g"].unpack_halo(s["st"][0], recv, mask=mask)
        for bk in blocks:
            s = sub[bk]
            s["g"].forward(s["st"], nt=1)
    torch.cuda.synchronize()
    out = np.zeros(shape)
    for bk in blocks:
        s = sub[bk]
        out[s["sl"]] = s["g"].domain(s["st"][0]).double().cpu().numpy()
    np.testing.assert_array_equal(out, ref)


# ---------------------------------------------------------------------------
# error paths that need a device
# ---------------------------------------------------------------------------

def test_model_above_vmax_is_rejected():
    FD = _fd()
    g = FD.Grid((16, 16, 16), (10.0,) * 3, 8, 1e-4, 2000.0)
    v = np.full((16, 16, 16), 1500.0, dtype=np.float32)
    v[3, 4, 5] = 2500.0
    with pytest.raises(FD.FdError) as e:
        g.set_model(to_dev(v))
    assert e.value.code == FD.FD_EUNSTABLE
    v[3, 4, 5] = -1.0
    with pytest.raises(FD.FdError):
        g.set_model(to_dev(v))


def test_receiver_outside_grid_is_rejected():
    FD = _fd()
    g = FD.Grid((16, 16, 16), (10.0,) * 3, 8, 1e-4, 2000.0)
    with pytest.raises(FD.FdError) as e:
        g.sparse(np.array([[10.0, 10.0, 150.5]]))
    assert e.value.code == FD.FD_EINVAL


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,so,tile", [((4, 5, 7), 8, None), ((6, 9, 70), 12, (8, 2, 1, 12)),
                                           ((4, 4), 8, None), ((4, 7, 130), 8, (4, 4, 3, 28))])
def test_grid_as_thin_as_the_stencil(shape, so, tile):
    """Axes as short as the stencil radius (the smallest the library
    accepts): neighbour reads reach across the whole axis into the zero
    halo, and sources/receivers on the first and last nodes (the clamped
    cell of the interpolation) behave as in the oracle."""
    rng = np.random.default_rng(21)
    h = (10.0,) * len(shape)
    vmax = 3000.0
    dt = synth.stable_dt(so, len(shape), 10.0, vmax)
    v = rng.uniform(1500.0, vmax, shape).astype(np.float32)
    last = [(s - 1) * 10.0 for s in shape]
    src = np.array([[0.0] * len(shape), last])
    rec = np.array([last, [0.0] * len(shape), [0.5 * x for x in last]])
    nt = 6
    q = (rng.standard_normal((nt, 2)) * 1e3).astype(np.float32)
    u0 = rng.standard_normal(shape).astype(np.float32)
    args = dict(shape=shape, spacing=h, so=so, dt=dt, vmax=vmax, v=v, nt=nt, src=src, q=q,
                rec=rec, u0=u0)
    gu, gum, gd = run_gpu_forward(tile=tile, **args)
    ou, oum, od = run_oracle_forward(**args)
    assert rel_l2(gu, ou) <= 1e-5
    assert rel_l2(gum, oum) <= 1e-5
    assert rel_l2(gd, od) <= 1e-5


def test_axis_shorter_than_the_stencil_radius_is_rejected():
    FD = _fd()
    with pytest.raises(FD.FdError):
        FD.Grid((3, 5, 7), (10.0,) * 3, 8, 1e-4, 3000.0)


def test_zero_steps_and_empty_sparse_sets():
    """nt = 0 leaves both states untouched; empty source and receiver sets
    are accepted and change nothing."""
    import torch
    FD = _fd()
    shape, so = (10, 12, 40), 8
    dt = synth.stable_dt(so, 3, 10.0, 3000.0)
    g = FD.Grid(shape, (10.0,) * 3, so, dt, 3000.0, nbl=3)
    g.set_model(to_dev(np.full(shape, 2000.0, np.float32)))
    rng = np.random.default_rng(22)
    a, b = g.field(), g.field()
    a.copy_(torch.from_numpy(rng.standard_normal(g.field_elems).astype(np.float32)))
    b.copy_(torch.from_numpy(rng.standard_normal(g.field_elems).astype(np.float32)))
    a0, b0 = a.clone(), b.clone()
    S = g.sparse(np.zeros((0, 3)))
    R = g.sparse(np.zeros((0, 3)))
    g.forward([a, b], S, torch.zeros((0, 0), device="cuda"), R,
              torch.zeros((0, 0), device="cuda"), 0)
    torch.cuda.synchronize()
    assert torch.equal(a, a0) and torch.equal(b, b0)
    # one update with empty sets equals one update without any
    c, e = a0.clone(), b0.clone()
    g.forward([a, b], S, torch.zeros((1, 0), device="cuda"), R,
              torch.zeros((1, 0), device="cuda"), 1)
    g.forward([c, e], nt=1)
    torch.cuda.synchronize()
    assert torch.equal(a, c) and torch.equal(b, e)
    g.close()


def test_autotune_json_cache(tmp_path):
    """The autotuner's JSON cache: a miss times the candidates and stores the
    winner under "arch|so|nz|ny|nx"; a second handle of the same shape gets
    the same tile from the cache without timing (ms 0) and then runs
    bit-identically to a handle given that tile explicitly; another shape is
    a miss again and both entries stay in the file."""
    import json
    FD = _fd()
    rng = np.random.default_rng(12)
    shape, so, h, vmax = (40, 36, 70), 8, 10.0, 3000.0
    v = synth.minmax(synth.smooth_noise(shape, 3.0, rng), 1500.0, vmax).astype(np.float32)
    dt = synth.stable_dt(so, 3, h, vmax)
    cache = str(tmp_path / "tiles.json")

    def tuned(shp, vv):
        g = FD.Grid(shp, (h,) * 3, so, dt, vmax, nbl=4)
        g.set_model(to_dev(vv))
        return g, g.autotune(cache)

    g1, (t1, ms1) = tuned(shape, v)
    assert ms1 > 0.0
    with open(cache) as f:
        entries = json.load(f)
    assert len(entries) == 1
    key, val = next(iter(entries.items()))
    assert key.endswith("|%d|%d|%d|%d" % ((so,) + shape)) and tuple(val) == tuple(t1)
    g1.close()
    g2, (t2, ms2) = tuned(shape, v)
    assert ms2 == 0.0 and tuple(t2) == tuple(t1)
    g2.close()
    u0 = synth.smooth_state(shape, 8, 3.0)
    a, _, _ = run_gpu_forward(shape, (h,) * 3, so, dt, vmax, v, 6, nbl=4, u0=u0, tile=tuple(t1))
    import torch
    g3, _ = tuned(shape, v)
    x, y = g3.field(), g3.field()
    g3.domain(x).copy_(to_dev(u0))
    g3.forward([x, y], nt=6)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g3.domain(x).double().cpu().numpy(), a)
    g3.close()
    shape2 = (24, 20, 70)
    v2 = synth.minmax(synth.smooth_noise(shape2, 3.0, rng), 1500.0, vmax).astype(np.float32)
    g4, (_, ms4) = tuned(shape2, v2)
    assert ms4 > 0.0
    g4.close()
    with open(cache) as f:
        assert len(json.load(f)) == 2
