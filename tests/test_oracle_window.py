"""Pin of the windowed oracle update that the full-size elastic and
visco-elastic GPU checks use: at points deep inside, inside the damping
layer and next to the faces of a periodic grid with a damping layer and a
fully three-dimensional medium, one update computed on the wrapped window
around each point equals the whole-grid oracle's update there.  Leaving out
the whole grid's damping rate, or clamping the window at the faces instead
of wrapping it, fails it."""
import numpy as np
import pytest

import oracle as O
import oracle.elastic as E
import oracle.visco as V
from paper_2312_13094_amd import synth
import window_oracle as W


def _setup(physics, seed):
    rng = np.random.default_rng(seed)
    n, so, nbl, h = 30, 4, 8, (10.0, 9.0, 11.0)
    shape = (n, n, n)
    vp = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 2000.0, 3500.0)
    vs = vp * synth.minmax(synth.smooth_noise(shape, 2.0, rng), 0.4, 0.6)
    rho = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 1600.0, 2600.0)
    dt = synth.elastic_stable_dt(so, min(h), 3600.0)
    g = O.Grid(shape, h, so=so, dt=dt, nbl=nbl, vmax=3600.0, bc=1)
    names = E.FIELDS if physics == "elastic" else V.FIELDS
    st = {f: g.zeros() for f in names}
    for f in names:
        g.interior(st[f])[...] = rng.standard_normal(shape) * (1e-3 if f[0] == "v" else 1e3)
    if physics == "elastic":
        med = (vp, vs, rho)
        coef = E.staggered_params(*E.medium(*med))
        whole, _ = E.forward(g, *med, nt=1, state=st)
    else:
        ts = synth.minmax(synth.smooth_noise(shape, 2.0, rng), 0.004, 0.008)
        tep = ts * synth.minmax(synth.smooth_noise(shape, 2.0, rng), 1.02, 1.1)
        tes = ts * synth.minmax(synth.smooth_noise(shape, 2.0, rng), 1.02, 1.2)
        med = (vp, vs, rho, tep, tes, ts)
        coef = V.coefficients(*med)
        whole, _ = V.forward(g, *med, nt=1, state=st)
    return rng, g, st, coef, whole, names


def _box(g, st, pt, names, wrap=True):
    """Padded window of half-width 3r around pt, from the DOMAIN values."""
    r = g.so // 2
    if wrap:
        idx = [W.wrapped(k, 3 * r, n) for k, n in zip(pt, g.shape)]
    else:       # clamped at the faces: what a window that ignores the wrap sees
        idx = [np.clip(np.arange(k - 3 * r, k + 3 * r + 1), 0, n - 1) for k, n in zip(pt, g.shape)]
    return {f: g.interior(st[f])[np.ix_(*idx)] for f in names}


@pytest.mark.parametrize("physics", ["elastic", "visco"])
def test_wrapped_window_with_global_damping_equals_whole_grid(physics):
    rng, g, st, coef, whole, names = _setup(physics, 61 if physics == "elastic" else 62)
    r = g.so // 2
    deep, layer, edge = W.sample_points(g.shape[0], g.nbl, r, rng, 6)
    mag = {f: np.abs(g.interior(whole[f])).max() for f in names}
    for pts in (deep, layer, edge):
        for pt in pts:
            got = W.step_at(g, physics, coef, _box(g, st, pt, names), pt)
            for f in names:
                want = g.interior(whole[f])[tuple(pt)]
                assert abs(got[f] - want) <= 1e-12 * mag[f], (physics, tuple(pt), f)
    # the checks bite: without the damping rate the layer points move, and a
    # window clamped at the faces gets the points next to them wrong
    flat = O.Grid(g.shape, g.spacing, so=g.so, dt=g.dt, nbl=0, vmax=g.vmax, bc=1)
    for pts, grid, wrap in ((layer, flat, True), (edge, g, False)):
        worst = 0.0
        for pt in pts:
            got = W.step_at(grid, physics, coef, _box(g, st, pt, names, wrap), pt)
            worst = max(worst, max(abs(got[f] - g.interior(whole[f])[tuple(pt)]) / mag[f]
                                   for f in names))
        assert worst > 1e-6, (physics, wrap)
