"""Pins of the TTI oracle: special cases that reduce to independently coded
operators, an exact discrete plane wave in a tilted medium, and the discrete
energy of the symmetrised system."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import tti as T
from paper_2312_13094_amd import synth
from test_oracle_pins import exact_d1


def _wide_second(u_pad, r, so, axis, h, n):
    """d/dx(d/dx u) with the exact first-derivative weights, the inner result
    extended by zero outside DOMAIN (coded here independently)."""
    a = [float(x) for x in exact_d1(so)]

    def d(upad):
        out = np.zeros(n)
        base = [slice(r, r + s) for s in n]
        for k in range(1, r + 1):
            p, m = list(base), list(base)
            p[axis] = slice(r + k, r + k + n[axis])
            m[axis] = slice(r - k, r - k + n[axis])
            out += a[k - 1] * (upad[tuple(p)] - upad[tuple(m)])
        return out / h

    inner = np.zeros(u_pad.shape)
    inner[tuple(slice(r, r + s) for s in n)] = d(u_pad)
    return d(inner)


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    sm = lambda: synth.smooth_noise(shape, 2.5, rng)
    return (synth.minmax(sm(), 1500, 3000), synth.minmax(sm(), 0.1, 0.3),
            synth.minmax(sm(), 0.0, 0.05), synth.minmax(sm(), 0, math.pi / 4),
            synth.minmax(sm(), 0, math.pi / 4))


@pytest.mark.parametrize("so", [4, 8, 12])
def test_isotropic_limit_any_tilt(so):
    """eps = delta = 0, p = r: H_xy + H_z = sum_i d_i d_i for any tilt field."""
    shape = (14, 13, 15)
    h = (10.0, 8.0, 12.0)
    g = O.Grid(shape, h, so=so, dt=1e-3)
    _, _, _, th, ph = _fields(shape, 1)
    u = g.pad(synth.smooth_state(shape, 2, 2.0).astype(np.float64))
    hxy, hz = T.operators(g, u, u, th, ph, 0)
    want = sum(_wide_second(u, g.r, so, ax, h[ax], shape) for ax in range(3))
    np.testing.assert_allclose(hxy + hz, want, rtol=0, atol=1e-12 * np.abs(want).max())


def _trilinear(coords, h, shape):
    """(node (z, y, x) index triples, weights) of each point's cell, coded
    here: base = floor(x / h) clamped to n - 2, weights the products of
    (1 - f) and f per axis."""
    out = []
    for c in np.asarray(coords, dtype=np.float64).reshape(-1, 3):
        base, frac = [], []
        for x, hh, n in zip(c, h, shape):
            b = min(int(math.floor(x / hh)), n - 2)
            base.append(b)
            frac.append(x / hh - b)
        nodes = []
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    wgt = ((frac[0] if bz else 1 - frac[0]) * (frac[1] if by else 1 - frac[1]) *
                           (frac[2] if bx else 1 - frac[2]))
                    nodes.append(((base[0] + bz, base[1] + by, base[2] + bx), wgt))
        out.append(nodes)
    return out


def test_isotropic_limit_forward_with_source_damping_receivers():
    """eps = delta = 0, p = r = 0 at the start, a source driving both fields:
    p and r stay equal to a time loop coded here independently, an acoustic
    forward whose Laplacian is the wide stencil sum_i d_i d_i (zero-extended
    intermediate), with u+ = [2u - (1-a)u- + v^2 dt^2 (L u + f)]/(1 + a),
    a = gamma dt / 2 from the acoustic damping profile, f the source spread
    by trilinear weights times q[n] / (hz hy hx), and receivers that sample
    p after each update.  A wrong source scale, damping factor or receiver
    time alignment in the TTI forward breaks the match."""
    shape, so, h, nbl, nt = (16, 15, 17), 8, (10.0, 9.0, 11.0), 4, 24
    v, _, _, th, ph = _fields(shape, 11)
    vmax = 3000.0
    dt = 0.4 * 2.0 / (vmax * math.sqrt(T.stability_number(so) * sum(1 / x ** 2 for x in h)))
    g = O.Grid(shape, h, so=so, dt=dt, nbl=nbl, vmax=vmax, bc=0)
    src = np.array([[73.0, 61.5, 93.5]])
    rec = np.array([[40.0, 30.0, 50.0], [101.0, 77.0, 130.0], [60.5, 100.0, 20.0]])
    q = (synth.ricker(nt, dt, 40.0)[:, None] * 1e3)
    zero = np.zeros(shape)
    p, _, r, _, d = T.forward(g, v, zero, zero, th, ph, src, q, rec, nt)
    # the loop coded here
    r_ = g.r
    gam = O.sponge_gamma(g)          # the acoustic damping profile (pinned separately)
    a = 0.5 * dt * gam
    v64 = np.asarray(v, dtype=np.float64)
    cvv = v64 * v64 * dt * dt
    snodes = _trilinear(src, h, shape)
    rnodes = _trilinear(rec, h, shape)
    u, um = g.zeros(), g.zeros()
    dref = np.zeros((nt, len(rec)))
    for n in range(nt):
        lap = sum(_wide_second(u, r_, so, ax, h[ax], shape) for ax in range(3))
        f = np.zeros(shape)
        for nodes in snodes:
            for idx, wgt in nodes:
                f[idx] += wgt * q[n, 0] / (h[0] * h[1] * h[2])
        un = (2 * g.interior(u) - (1 - a) * g.interior(um) + cvv * (lap + f)) / (1 + a)
        um, u = u, g.pad(un)
        for i, nodes in enumerate(rnodes):
            dref[n, i] = sum(wgt * un[idx] for idx, wgt in nodes)
    scale = np.abs(g.interior(u)).max()
    assert scale > 0
    np.testing.assert_allclose(g.interior(p), g.interior(u), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(g.interior(r), g.interior(u), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(d, dref, rtol=0, atol=1e-12 * np.abs(dref).max())
    assert np.abs(dref).max() > 0


def test_vertical_axis_is_vti():
    """theta = 0: H_z = d_z d_z and H_xy = d_x d_x + d_y d_y (any phi)."""
    shape, so, h = (12, 14, 13), 8, (10.0, 9.0, 11.0)
    g = O.Grid(shape, h, so=so, dt=1e-3)
    p = g.pad(synth.smooth_state(shape, 3, 2.0).astype(np.float64))
    r = g.pad(synth.smooth_state(shape, 4, 2.0).astype(np.float64))
    zero = np.zeros(shape)
    hxy, hz = T.operators(g, p, r, zero, zero + 0.7, 0)
    np.testing.assert_allclose(hz, _wide_second(r, g.r, so, 0, h[0], shape), atol=1e-11)
    want = _wide_second(p, g.r, so, 1, h[1], shape) + _wide_second(p, g.r, so, 2, h[2], shape)
    np.testing.assert_allclose(hxy, want, atol=1e-11)


def test_tilted_plane_wave_is_exact():
    """Periodic homogeneous tilted medium: cos(k.x - w t) times an eigenvector
    of the 2x2 symbol is an exact discrete solution.  With s_j the symbol of
    the first derivative, A = |s|^2 - (a.s)^2, B = (a.s)^2 and the textbook
    axis a = (sin t cos f, sin t sin f, cos t), the pair (p, r) obeys
    q_tt = -v^2 [[(1+2e) A, sqrt(1+2d) B], [sqrt(1+2d) A, B]] q."""
    shape, so = (16, 18, 20), 8
    h = (10.0, 12.0, 9.0)
    v, e, d, th, ph = 2000.0, 0.2, 0.05, 0.6, 0.4
    a1 = [float(x) for x in exact_d1(so)]
    modes = (1, 2, 3)
    kk = [2 * math.pi * m / (n * hh) for m, n, hh in zip(modes, shape, h)]
    s = [2.0 / hh * sum(a1[j - 1] * math.sin(j * k * hh) for j in range(1, so // 2 + 1))
         for k, hh in zip(kk, h)]
    axis = (math.cos(th), math.sin(th) * math.sin(ph), math.sin(th) * math.cos(ph))  # (z,y,x)
    as_ = sum(ai * si for ai, si in zip(axis, s))
    A = sum(si * si for si in s) - as_ ** 2
    B = as_ ** 2
    M = np.array([[(1 + 2 * e) * A, math.sqrt(1 + 2 * d) * B], [math.sqrt(1 + 2 * d) * A, B]])
    lam, vec = np.linalg.eig(M)
    i = int(np.argmax(lam.real))
    lam, vec = lam[i].real, vec[:, i].real
    dt = 0.3 * 2.0 / (v * math.sqrt(lam))
    om = 2 * math.asin(math.sqrt(v * v * dt * dt * lam / 4)) / dt
    g = O.Grid(shape, h, so=so, dt=dt, bc=1)
    xs = np.meshgrid(*[np.arange(n) * hh for n, hh in zip(shape, h)], indexing="ij")
    phase = sum(k * x for k, x in zip(kk, xs))
    P, R = vec
    full = lambda f: np.full(shape, f)
    nt = 120
    p, _, r, _, _ = T.forward(g, full(v), full(e), full(d), full(th), full(ph), nt=nt,
                              p0=g.pad(P * np.cos(phase)), pm=g.pad(P * np.cos(phase + om * dt)),
                              r0=g.pad(R * np.cos(phase)), rm=g.pad(R * np.cos(phase + om * dt)))
    want = np.cos(phase - om * nt * dt)
    assert np.abs(g.interior(p) - P * want).max() < 1e-10
    assert np.abs(g.interior(r) - R * want).max() < 1e-10


def test_energy_of_symmetrised_system_is_conserved():
    """Zero halo, no damping, no source, eps > delta: with K = v^2 [[1+2e,
    sqrt(1+2d)], [sqrt(1+2d), 1]] (pointwise SPD) and H = diag(H_xy, H_z)
    (symmetric), E = 1/2 <dq, K^-1 dq>/dt^2 - 1/2 <q+, H q> is constant."""
    shape, so, h = (16, 15, 17), 8, (10.0, 10.0, 10.0)
    v, e, d, th, ph = _fields(shape, 5)
    S1 = T.stability_number(so)
    dt = 0.4 * 2.0 / (3000.0 * math.sqrt(1.6) * math.sqrt(S1 * 3 / 100.0))
    g = O.Grid(shape, h, so=so, dt=dt, bc=0)
    taper = np.pad(np.ones(tuple(s - 8 for s in shape)), 4)
    p = g.pad(synth.smooth_state(shape, 6, 2.0).astype(np.float64) * taper)
    r = g.pad(synth.smooth_state(shape, 7, 2.0).astype(np.float64) * taper)
    pm, rm = p.copy(), r.copy()
    c12 = np.sqrt(1 + 2 * d)
    det = (1 + 2 * e) - c12 ** 2
    es = []
    for _ in range(40):
        pn, po, rn, ro, _ = T.forward(g, v, e, d, th, ph, nt=1, p0=p, pm=pm, r0=r, rm=rm)
        hxy, hz = T.operators(g, po, ro, th, ph, 0)
        dp = (g.interior(pn) - g.interior(po)) / dt
        dr = (g.interior(rn) - g.interior(ro)) / dt
        kin = 0.5 * np.sum((dp * dp - 2 * c12 * dp * dr + (1 + 2 * e) * dr * dr) / (det * v * v))
        pot = -0.5 * (np.sum(g.interior(pn) * hxy) + np.sum(g.interior(rn) * hz))
        es.append(kin + pot)
        p, pm, r, rm = pn, po, rn, ro
    es = np.array(es)
    assert np.abs(es - es[0]).max() <= 1e-11 * abs(es[0])


def test_stability_number():
    """S1 for so 12 (3.6897) from the symbol's peak; so 2 gives 1."""
    assert abs(T.stability_number(2) - 1.0) < 1e-9
    assert abs(T.stability_number(12) - 3.6897) < 1e-3


def _window(n, k, w):
    """Index box of half-width w around k, clipped at the DOMAIN faces."""
    lo = tuple(max(int(c) - w, 0) for c in k)
    hi = tuple(min(int(c) + w + 1, s) for c, s in zip(k, n))
    return lo, hi


def test_clipped_window_with_global_damping_equals_whole_grid():
    """The windowed oracle the 384^3 GPU check uses: one step at a point from
    a window of half-width 2R around it, clipped at the DOMAIN faces (where
    the window's zero halo is the grid's own) and carrying the whole grid's
    damping rate (sponge_gamma_box), equals the whole-grid step there, for
    points deep inside, inside the damping layer and next to the faces.  A
    window of half-width R, or one without the whole grid's damping rate,
    fails it."""
    shape, so, nbl, h = (26, 24, 28), 6, 5, (10.0, 10.0, 10.0)
    R = so // 2
    rng = np.random.default_rng(31)
    F = {k: rng.uniform(lo, hi, shape) for k, lo, hi in
         [("v", 1500, 4500), ("eps", 0, 0.3), ("delta", 0, 0.15),
          ("theta", 0, math.pi / 4), ("phi", 0, math.pi / 4)]}
    dt = 0.4 * 2.0 / (4500 * math.sqrt(1.6) * math.sqrt(T.stability_number(so) * 3 / 100.0))
    g = O.Grid(shape, h, so=so, dt=dt, nbl=nbl, vmax=4500.0, bc=0)
    init = [rng.standard_normal(shape) for _ in range(4)]
    whole = T.forward(g, F["v"], F["eps"], F["delta"], F["theta"], F["phi"], nt=1,
                      p0=g.pad(init[0]), pm=g.pad(init[1]), r0=g.pad(init[2]),
                      rm=g.pad(init[3]))
    gam = O.sponge_gamma(g)
    pts = [(13, 12, 14), (2, 12, 14), (13, 21, 3), (0, 0, 27), (25, 23, 0), (7, 1, 22)]
    for k in pts:
        lo, hi = _window(shape, k, 2 * R)
        win = tuple(slice(a, b) for a, b in zip(lo, hi))
        gw = O.sponge_gamma_box(g, lo, hi)
        np.testing.assert_array_equal(gw, gam[win])
        og = O.Grid(tuple(b - a for a, b in zip(lo, hi)), h, so=so, dt=dt, nbl=0,
                    vmax=4500.0, bc=0)
        p, _, r, _, _ = T.forward(og, F["v"][win], F["eps"][win], F["delta"][win],
                                  F["theta"][win], F["phi"][win], nt=1,
                                  p0=og.pad(init[0][win]), pm=og.pad(init[1][win]),
                                  r0=og.pad(init[2][win]), rm=og.pad(init[3][win]), gamma=gw)
        c = tuple(a - b for a, b in zip(k, lo))
        for got, want in ((og.interior(p)[c], g.interior(whole[0])[k]),
                          (og.interior(r)[c], g.interior(whole[2])[k])):
            assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (k, got, want)
