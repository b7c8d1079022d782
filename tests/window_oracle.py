"""Windowed oracle updates for sampled checks of full-size launches.

One velocity-stress update at a DOMAIN point depends only on the fields
within 2r cells of it (the stress at the point reads velocities within r,
and those read stresses within r more) and on the medium within r + 1.  So
the oracle's two half steps (Virieux's staggered scheme; the visco-elastic
one adds the memory variables of one standard linear solid), run on the
window of half-width 2r around the point with a halo of r more, give the
whole grid's value there.  The window is taken with wrapped indices (the
periodic halo of the grid), its medium coefficients are the whole grid's at
those indices (so the grid's own treatment of the last DOMAIN index holds)
and its damping rate is the whole grid's (sponge_gamma_at), which makes the
procedure valid deep inside, in the damping layer and next to the faces.
Test infrastructure: it calls only the oracle."""
import numpy as np

import oracle as O
import oracle.elastic as E
import oracle.visco as V


def wrapped(k, w, n):
    """DOMAIN indices k - w .. k + w along one axis of size n, wrapped."""
    return np.arange(int(k) - w, int(k) + w + 1) % n


def _take(coef, idx, sub):
    """Whole-grid coefficient arrays (each axis of size n or 1) at the
    window's indices, broadcast to the window."""
    out = {}
    for name, v in coef.items():
        v = np.asarray(v, dtype=np.float64)
        sel = np.ix_(*(i if m > 1 else [0] for i, m in zip(idx, v.shape)))
        out[name] = np.broadcast_to(v[sel], sub)
    return out


def step_at(big: O.Grid, physics: str, coef, box, pt):
    """Values of every component at DOMAIN point pt of the periodic grid big
    after one update.  physics: "elastic" (coef from
    E.staggered_params(*E.medium(...))) or "visco" (coef from
    V.coefficients(...)), computed on the whole grid; box maps each field
    name to its padded window, the (6r + 1)^3 values at wrapped indices
    around pt (half-width 3r)."""
    r = big.so // 2
    w = 2 * r
    sub = (2 * w + 1,) * 3
    og = O.Grid(sub, big.spacing, so=big.so, dt=big.dt)
    idx = [wrapped(k, w, n) for k, n in zip(pt, big.shape)]
    par = _take(coef, idx, sub)
    a = 0.5 * big.dt * O.sponge_gamma_at(big, *idx)
    names = E.FIELDS if physics == "elastic" else V.FIELDS
    st = {name: np.array(box[name], dtype=np.float64) for name in names}
    if physics == "elastic":
        E.velocity_update(og, st, par, a)
        E.stress_update(og, st, par, a)
    else:
        E.velocity_update(og, st, {k: par[k] for k in ("bx", "by", "bz")}, a)
        V.stress_memory_update(og, st, par, a)
    return {name: float(og.interior(st[name])[w, w, w]) for name in names}


def sample_points(n, nbl, r, rng, count):
    """count points each deep inside (beyond the damping layer and 3r
    more), inside the damping layer (3r or more from the faces) and within 3r
    of a face (cycling over the six faces), as three (count, 3) arrays."""
    w = 3 * r
    deep = rng.integers(nbl + w, n - nbl - w, size=(count, 3))
    layer = rng.integers(0, n, size=(count, 3))
    edge = rng.integers(0, n, size=(count, 3))
    for i in range(count):
        ax, hi_side = i % 3, (i // 3) % 2
        d = int(rng.integers(w, nbl))
        layer[i, ax] = n - 1 - d if hi_side else d
        e = int(rng.integers(0, w))
        edge[i, ax] = n - 1 - e if hi_side else e
    return deep, layer, edge
