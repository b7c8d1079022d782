"""Pins of the FP64 elastic oracle against what the mathematics fixes:
published staggered-grid weights, polynomial exactness, exact discrete plane
waves of the periodic homogeneous medium (all nine components, P and S),
conservation of the scheme's discrete energy in heterogeneous media, the
closed-form first update of a source, and mirror symmetry."""
import math

import numpy as np
import pytest
from fractions import Fraction

import oracle as O
import oracle.elastic as E
from paper_2312_13094_amd import synth


def test_staggered_weights_match_published_values():
    # second-, fourth- and eighth-order staggered first-derivative weights
    # (Levander 1988; Fornberg's tables)
    assert E.staggered_weights_exact(2) == [Fraction(1)]
    assert E.staggered_weights_exact(4) == [Fraction(9, 8), Fraction(-1, 24)]
    assert E.staggered_weights_exact(8) == [Fraction(1225, 1024), Fraction(-245, 3072),
                                            Fraction(49, 5120), Fraction(-5, 7168)]


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16])
def test_cfl_table_matches_weights(so):
    """The time-step table of the input generator agrees with the weights."""
    assert synth._STAG[so] == pytest.approx(E.cfl_number(so), rel=1e-14)


@pytest.mark.parametrize("so", [4, 8, 12])
@pytest.mark.parametrize("ax", [0, 1, 2])
def test_staggered_derivatives_exact_on_polynomials(so, ax):
    """Dp / Dm of a polynomial of degree 2r equal its derivative at the half
    point / node (the odd Taylor terms beyond degree 2r are absent)."""
    r = so // 2
    shape = [3, 3, 3]
    shape[ax] = 10
    h = [10.0, 7.0, 5.0]
    g = O.Grid(tuple(shape), tuple(h), so=so, dt=1e-3)
    rng = np.random.default_rng(so + 10 * ax)
    coef = rng.standard_normal(2 * r + 1)
    L = (shape[ax] + 2 * r) * h[ax]
    P = np.polynomial.Polynomial(coef)
    dP = P.deriv()

    def along(vals):
        sh = [1, 1, 1]
        sh[ax] = -1
        return np.broadcast_to(vals.reshape(sh), g.padded_shape).copy()

    xs = (np.arange(shape[ax] + 2 * r) - r) * h[ax]
    node = along(P(xs / L))
    half = along(P((xs + 0.5 * h[ax]) / L))
    dom = np.arange(shape[ax]) * h[ax]
    want_half = dP((dom + 0.5 * h[ax]) / L) / L
    want_node = dP(dom / L) / L
    sl = [0, 0, 0]
    sl[ax] = slice(None)
    got_p = E.dplus(g, node, ax)[tuple(sl)]
    got_m = E.dminus(g, half, ax)[tuple(sl)]
    scale = np.abs(want_node).max()
    np.testing.assert_allclose(got_p, want_half, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(got_m, want_node, rtol=0, atol=1e-9 * scale)


def test_staggered_params_are_midpoint_values_of_linear_media():
    """Averaging over the nodes around a staggered point gives the exact
    midpoint value of a medium linear (bilinear) in the averaged axes."""
    z, y, x = np.meshgrid(np.arange(6.0), np.arange(7.0), np.arange(8.0), indexing="ij")
    b = 1.0 + 0.1 * x - 0.05 * y + 0.02 * z
    mu = 2.0 + 0.3 * y + 0.2 * x + 0.05 * x * y + 0.1 * z + 0.07 * z * x + 0.03 * z * y
    lam = 3.0 + 0 * x
    p = E.staggered_params(b, lam, mu)
    inner = (slice(0, 5), slice(0, 6), slice(0, 7))

    def bf(z, y, x):
        return 1.0 + 0.1 * x - 0.05 * y + 0.02 * z

    def muf(z, y, x):
        return 2.0 + 0.3 * y + 0.2 * x + 0.05 * x * y + 0.1 * z + 0.07 * z * x + 0.03 * z * y

    np.testing.assert_allclose(p["bx"][inner], bf(z, y, x + 0.5)[inner], rtol=1e-14)
    np.testing.assert_allclose(p["by"][inner], bf(z, y + 0.5, x)[inner], rtol=1e-14)
    np.testing.assert_allclose(p["bz"][inner], bf(z + 0.5, y, x)[inner], rtol=1e-14)
    np.testing.assert_allclose(p["mxy"][inner], muf(z, y + 0.5, x + 0.5)[inner], rtol=1e-14)
    np.testing.assert_allclose(p["mxz"][inner], muf(z + 0.5, y, x + 0.5)[inner], rtol=1e-14)
    np.testing.assert_allclose(p["myz"][inner], muf(z + 0.5, y + 0.5, x)[inner], rtol=1e-14)
    # beyond DOMAIN the last node value repeats
    np.testing.assert_allclose(p["bx"][:, :, -1], b[:, :, -1], rtol=1e-15)


NAMES = {0: "z", 1: "y", 2: "x"}


def _vel_name(pol):
    return "v" + NAMES[pol]


def _stress_name(a, b):
    order = {2: 0, 1: 1, 0: 2}          # x, y, z in component names
    i, j = sorted((a, b), key=lambda t: order[t])
    return "t" + NAMES[i] + NAMES[j]


@pytest.mark.parametrize("so", [4, 8])
@pytest.mark.parametrize("ax,pol", [(a, p) for a in range(3) for p in range(3)])
def test_discrete_plane_waves_are_exact(so, ax, pol):
    """Periodic homogeneous medium: the discrete plane wave
    tau = T cos(k x - w t), v = -T / (rho c) cos(k x' - w t') with
    sin(w dt / 2) = (dt / 2) c K(k), K = (2 / h) sum_k c_k sin((2k - 1) k h / 2)
    (c = vp for P, pol == ax; c = vs for S) is reproduced to rounding."""
    r = so // 2
    shape = [max(5, r + 1)] * 3
    shape[ax] = 24
    h = [10.0, 8.0, 12.0]
    vp, vs, rho = 3000.0, 1700.0, 2200.0
    dt = synth.elastic_stable_dt(so, min(h), vp, frac=0.8)
    g = O.Grid(tuple(shape), tuple(h), so=so, dt=dt, bc=1)
    lam, mu = rho * (vp * vp - 2 * vs * vs), rho * vs * vs
    c = vp if ax == pol else vs
    kw = 2 * math.pi * 3 / (shape[ax] * h[ax])
    cw = E.staggered_weights(so)
    K = 2.0 / h[ax] * sum(cw[k - 1] * math.sin((2 * k - 1) * kw * h[ax] / 2) for k in range(1, r + 1))
    w = 2.0 / dt * math.asin(dt / 2 * c * K)
    idx = np.arange(shape[ax]) * h[ax]

    def along(vals):
        sh = [1, 1, 1]
        sh[ax] = -1
        return np.broadcast_to(vals.reshape(sh), g.shape)

    # stress at the node along ax for P (normal stresses), at the half point
    # for S (the shear stress is staggered along ax); velocity the other way
    xs_t = idx if ax == pol else idx + 0.5 * h[ax]
    xs_v = idx + 0.5 * h[ax] if ax == pol else idx

    def fields(n_t, n_v):
        st = E.zero_state(g)
        T = np.cos(kw * xs_t - w * n_t * dt)
        V = -np.cos(kw * xs_v - w * n_v * dt) / (rho * c)
        if ax == pol:
            for a in range(3):
                ratio = 1.0 if a == ax else lam / (lam + 2 * mu)
                g.interior(st[_stress_name(a, a)])[...] = along(ratio * T)
        else:
            g.interior(st[_stress_name(ax, pol)])[...] = along(T)
        g.interior(st[_vel_name(pol)])[...] = along(V)
        return st

    nt = 17
    s0 = fields(0, -0.5)
    full = (lambda v: np.full(tuple(shape), v))
    got, _ = E.forward(g, full(vp), full(vs), full(rho), nt=nt, state=s0)
    want = fields(nt, nt - 0.5)
    for f in E.FIELDS:
        np.testing.assert_allclose(g.interior(got[f]), g.interior(want[f]), rtol=0, atol=1e-11,
                                   err_msg=f)
    # the wave actually moved (not a trivial pass)
    v0 = g.interior(s0[_vel_name(pol)])
    assert np.abs(g.interior(want[_vel_name(pol)]) - v0).max() > 0.1 * np.abs(v0).max()


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("so", [4, 8])
def test_energy_is_conserved_in_heterogeneous_media(bc, so):
    """Without damping the staggered leapfrog conserves
    1/2 <v^(n+1/2), v^(n-1/2)>_(1/b) + 1/2 <tau^n, C^-1 tau^n> exactly (the
    discrete divergence and strain rate are negative adjoints), for any
    positive medium, with zero or periodic halos."""
    rng = np.random.default_rng(7 + so + bc)
    shape, h = (11, 10, 12), (9.0, 10.0, 11.0)
    vp = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 2000.0, 3500.0)
    vs = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 800.0, 1500.0)
    rho = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 1500.0, 2600.0)
    dt = synth.elastic_stable_dt(so, min(h), 3500.0, frac=0.9)
    g = O.Grid(shape, h, so=so, dt=dt, bc=bc)
    par = E.staggered_params(*E.medium(vp, vs, rho))
    s = E.zero_state(g)
    for f in E.FIELDS:
        g.interior(s[f])[...] = rng.standard_normal(shape)
    a = np.zeros(shape)
    es = []
    for _ in range(30):
        for f in E.FIELDS[3:]:
            E._fill(g, s[f], bc)
        v_old = {f: s[f].copy() for f in E.FIELDS[:3]}
        E.velocity_update(g, s, par, a)
        es.append(E.energy(g, v_old, s, s, par))
        for f in E.FIELDS[:3]:
            E._fill(g, s[f], bc)
        E.stress_update(g, s, par, a)
    es = np.array(es)
    assert np.abs(es - es[0]).max() <= 1e-12 * abs(es[0])
    # and a wrong placement breaks it: mu at nodes for the shear stresses
    bad = dict(par, mxy=par["mu"], mxz=par["mu"], myz=par["mu"])
    s2 = E.zero_state(g)
    for f in E.FIELDS:
        g.interior(s2[f])[...] = rng.standard_normal(shape)
    e2 = []
    for _ in range(30):
        for f in E.FIELDS[3:]:
            E._fill(g, s2[f], bc)
        v_old = {f: s2[f].copy() for f in E.FIELDS[:3]}
        E.velocity_update(g, s2, bad, a)
        e2.append(E.energy(g, v_old, s2, s2, par))
        for f in E.FIELDS[:3]:
            E._fill(g, s2[f], bc)
        E.stress_update(g, s2, bad, a)
    e2 = np.array(e2)
    assert np.abs(e2 - e2[0]).max() > 1e-6 * abs(e2[0])


def test_first_update_of_a_source_is_closed_form():
    """From rest, one update leaves v = 0 and adds dt q w / h^3 to each normal
    stress at the source's eight nodes (multilinear weights), nothing else;
    the receiver at the source then reads 3 sum_c w_c^2 dt q / h^3."""
    shape, h, so = (9, 10, 11), (10.0, 8.0, 12.0), 8
    dt = 1e-3
    g = O.Grid(shape, h, so=so, dt=dt)
    pos = np.array([[3.25 * h[0], 4.5 * h[1], 5.75 * h[2]]])
    q = np.array([[2.5]])
    full = (lambda v: np.full(shape, v))
    s, d = E.forward(g, full(3000.0), full(1500.0), full(2000.0), src=pos, q=q, rec=pos, nt=1)
    wz, wy, wx = {3: 0.75, 4: 0.25}, {4: 0.5, 5: 0.5}, {5: 0.25, 6: 0.75}
    want = np.zeros(shape)
    for z, a in wz.items():
        for y, b in wy.items():
            for x, c in wx.items():
                want[z, y, x] = dt * 2.5 * a * b * c / (h[0] * h[1] * h[2])
    for f in ("txx", "tyy", "tzz"):
        np.testing.assert_allclose(g.interior(s[f]), want, rtol=1e-14, atol=0)
    for f in ("vx", "vy", "vz", "txy", "txz", "tyz"):
        assert not g.interior(s[f]).any()
    assert d[0, 0] == pytest.approx(3 * np.sum(want * want) / (dt * 2.5 / np.prod(h)), rel=1e-14)


def test_mirror_symmetry_under_x_y_exchange():
    """A medium and a source symmetric under x <-> y (equal spacing) give
    fields with vx(z, y, x) = vy(z, x, y), txx = tyy^T, txz = tyz^T and vz,
    tzz, txy symmetric (the staggered positions map onto each other),
    damping layer included."""
    n, nz, so = 14, 12, 8
    h = (9.0, 10.0, 10.0)
    rng = np.random.default_rng(3)

    def sym(a):
        return 0.5 * (a + a.transpose(0, 2, 1))

    vp = sym(synth.minmax(synth.smooth_noise((nz, n, n), 2.0, rng), 2000.0, 3000.0))
    vs = sym(synth.minmax(synth.smooth_noise((nz, n, n), 2.0, rng), 900.0, 1400.0))
    rho = sym(synth.minmax(synth.smooth_noise((nz, n, n), 2.0, rng), 1800.0, 2400.0))
    dt = synth.elastic_stable_dt(so, 9.0, 3000.0)
    g = O.Grid((nz, n, n), h, so=so, dt=dt, nbl=3, vmax=3000.0)
    src = np.array([[5.3 * h[0], 6.4 * h[1], 6.4 * h[2]]])
    q = synth.ricker(30, dt, 40.0, t0=0.01)[:, None].astype(np.float64) * 1e3
    s, _ = E.forward(g, vp, vs, rho, src=src, q=q, nt=30)
    I = g.interior

    def T(a):
        return a.transpose(0, 2, 1)

    scale = max(np.abs(I(s[f])).max() for f in E.FIELDS)
    assert scale > 0
    tol = dict(rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(I(s["vx"]), T(I(s["vy"])), **tol)
    np.testing.assert_allclose(I(s["txx"]), T(I(s["tyy"])), **tol)
    np.testing.assert_allclose(I(s["txz"]), T(I(s["tyz"])), **tol)
    for f in ("vz", "tzz", "txy"):
        np.testing.assert_allclose(I(s[f]), T(I(s[f])), **tol)
    # the mirror does not hold for a source off the diagonal
    s2, _ = E.forward(g, vp, vs, rho, src=src + np.array([[0, 2 * h[1], 0]]), q=q, nt=30)
    assert np.abs(I(s2["vx"]) - T(I(s2["vy"]))).max() > 0.01 * np.abs(I(s2["vx"])).max()


@pytest.mark.parametrize("frac,grows", [(0.99, False), (1.02, True)])
def test_cfl_limit_of_the_checkerboard_mode(frac, grows):
    """The highest mode (checkerboard along every axis, an S-free P mode of
    the periodic homogeneous medium) stays bounded just below
    vp dt sqrt(sum 1/h^2) sum|c_k| = 1 and grows just above it."""
    so, shape, h = 8, (8, 8, 8), (10.0, 10.0, 10.0)
    vp, vs, rho = 3000.0, 0.0, 2000.0
    dt = frac / (vp * math.sqrt(3.0) / h[0] * E.cfl_number(so))
    g = O.Grid(shape, h, so=so, dt=dt, bc=1)
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    st = E.zero_state(g)
    chk = (-1.0) ** (z + y + x)
    for f in ("txx", "tyy", "tzz"):
        g.interior(st[f])[...] = chk
    full = (lambda v: np.full(shape, v))
    s, _ = E.forward(g, full(vp), full(vs), full(rho), nt=400, state=st)
    amp = max(np.abs(g.interior(s[f])).max() for f in ("txx", "tyy", "tzz"))
    assert (amp > 10.0) == grows
