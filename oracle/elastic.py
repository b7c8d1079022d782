"""FP64 oracle of the isotropic elastic velocity-stress step (test
infrastructure only: tests, smoke() and bench.py's CPU baseline use it; the
HIP path never does).

Paper, appendix "Isotropic elastic", equation (elas1): with buoyancy
b = 1/rho and the Lame parameters lambda, mu,

    v_t   = b div(tau)
    tau_t = lambda tr(grad v) I + mu (grad v + grad v^T)

a first-order system in time with nine wavefield components.  The paper
prints no discretisation (it cites Virieux 1986); the reading used here is
Virieux's staggered grid:

* storage index (z, y, x) holds each component at its own position:
  vx (z, y, x+1/2), vy (z, y+1/2, x), vz (z+1/2, y, x);
  txx, tyy, tzz at the node (z, y, x);
  txy (z, y+1/2, x+1/2), txz (z+1/2, y, x+1/2), tyz (z+1/2, y+1/2, x);
* staggered first derivatives of order so with r = so/2 weights c_k:
    Dp f[i] = sum_k c_k (f[i+k] - f[i-k+1]) / h   (node -> half point)
    Dm f[i] = sum_k c_k (f[i+k-1] - f[i-k]) / h   (half point -> node)
  c_k make the difference exact for polynomials of degree <= 2r;
* time staggered: v at half steps from tau^n, then tau^(n+1) from the new v;
* the medium at a component's position: b averaged over the two nodes along
  the velocity's staggered axis; mu averaged over the four nodes of a shear
  stress's staggered plane; lambda, mu at nodes for the normal stresses;
  node values beyond DOMAIN repeat the last DOMAIN value;
* damping as in the acoustic scheme, per component at its storage index:
  w+ = [(1 - a) w + dt rhs] / (1 + a), a = gamma dt / 2;
* an explosive source: q(t) delta(x - x_s) added to the rate of each normal
  stress, i.e. txx, tyy, tzz += dt w q / (h^3 (1 + a)) at the source's eight
  nodes after update n (multilinear weights w, q[n]);
* receivers record txx + tyy + tzz at their nodes after each update.

Halos: zero (bc 0) or periodic (bc 1), filled before each half step.
Arrays are (z, y, x); padded fields carry a halo of r = so/2.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import Grid, sparse_weights, sponge_gamma
from .tti import _fill

FIELDS = ("vx", "vy", "vz", "txx", "tyy", "tzz", "txy", "txz", "tyz")
Z, Y, X = 0, 1, 2


def staggered_weights_exact(so: int):
    """c_1..c_r as Fractions: sum_k c_k (2k-1)^(2m-1) = [m == 1], m = 1..r
    (Taylor expansion of f(+(k-1/2)h) - f(-(k-1/2)h) about the midpoint)."""
    if so < 2 or so % 2:
        raise ValueError("bad space order %r" % so)
    r = so // 2
    A = [[Fraction((2 * k - 1) ** (2 * m - 1)) for k in range(1, r + 1)] for m in range(1, r + 1)]
    b = [Fraction(1 if m == 1 else 0) for m in range(1, r + 1)]
    # Gaussian elimination in exact arithmetic
    for i in range(r):
        piv = next(j for j in range(i, r) if A[j][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        b[i], b[piv] = b[piv], b[i]
        for j in range(r):
            if j != i and A[j][i] != 0:
                f = A[j][i] / A[i][i]
                A[j] = [x - f * y for x, y in zip(A[j], A[i])]
                b[j] -= f * b[i]
    return [b[i] / A[i][i] for i in range(r)]


def staggered_weights(so: int) -> np.ndarray:
    return np.array([float(c) for c in staggered_weights_exact(so)])


def _shift(g: Grid, f: np.ndarray, ax: int, s: int) -> np.ndarray:
    """DOMAIN-shaped view of padded f displaced by s along axis ax."""
    r = g.r
    sl = [slice(r, r + n) for n in g.shape]
    sl[ax] = slice(r + s, r + s + g.shape[ax])
    return f[tuple(sl)]


def dplus(g: Grid, f: np.ndarray, ax: int) -> np.ndarray:
    """Derivative at i + 1/2 along ax of node-positioned f (padded)."""
    c = staggered_weights(g.so)
    out = np.zeros(g.shape)
    for k in range(1, g.r + 1):
        out += c[k - 1] * (_shift(g, f, ax, k) - _shift(g, f, ax, -(k - 1)))
    return out / g.spacing[ax]


def dminus(g: Grid, f: np.ndarray, ax: int) -> np.ndarray:
    """Derivative at the node along ax of half-point-positioned f (padded)."""
    c = staggered_weights(g.so)
    out = np.zeros(g.shape)
    for k in range(1, g.r + 1):
        out += c[k - 1] * (_shift(g, f, ax, k - 1) - _shift(g, f, ax, -k))
    return out / g.spacing[ax]


def _next(m: np.ndarray, ax: int) -> np.ndarray:
    """m at index i + 1 along ax, the last DOMAIN value repeated."""
    idx = np.minimum(np.arange(m.shape[ax]) + 1, m.shape[ax] - 1)
    return np.take(m, idx, axis=ax)


def medium(vp, vs, rho):
    """Node values (b, lambda, mu) from velocities and density."""
    vp, vs, rho = (np.asarray(a, dtype=np.float64) for a in (vp, vs, rho))
    mu = rho * vs * vs
    return 1.0 / rho, rho * vp * vp - 2.0 * mu, mu


def staggered_params(b, lam, mu):
    """The medium at each component's position: dict of DOMAIN arrays
    bx, by, bz (velocities), lam, mu (normal stresses), mxy, mxz, myz."""
    out = {"bx": 0.5 * (b + _next(b, X)), "by": 0.5 * (b + _next(b, Y)),
           "bz": 0.5 * (b + _next(b, Z)), "lam": lam, "mu": mu}
    for name, (p, q) in (("mxy", (Y, X)), ("mxz", (Z, X)), ("myz", (Z, Y))):
        out[name] = 0.25 * (mu + _next(mu, p) + _next(mu, q) + _next(_next(mu, p), q))
    return out


def velocity_update(g: Grid, s, par, a):
    """v^(n+1/2) from v^(n-1/2) and tau^n (halos of tau filled)."""
    dt = g.dt
    rhs = {
        "vx": dplus(g, s["txx"], X) + dminus(g, s["txy"], Y) + dminus(g, s["txz"], Z),
        "vy": dminus(g, s["txy"], X) + dplus(g, s["tyy"], Y) + dminus(g, s["tyz"], Z),
        "vz": dminus(g, s["txz"], X) + dminus(g, s["tyz"], Y) + dplus(g, s["tzz"], Z),
    }
    for f, bname in (("vx", "bx"), ("vy", "by"), ("vz", "bz")):
        g.interior(s[f])[...] = ((1.0 - a) * g.interior(s[f]) +
                                 dt * par[bname] * rhs[f]) / (1.0 + a)


def stress_update(g: Grid, s, par, a):
    """tau^(n+1) from tau^n and v^(n+1/2) (halos of v filled)."""
    dt = g.dt
    e = {"txx": dminus(g, s["vx"], X), "tyy": dminus(g, s["vy"], Y),
         "tzz": dminus(g, s["vz"], Z)}
    tr = e["txx"] + e["tyy"] + e["tzz"]
    rhs = {f: par["lam"] * tr + 2.0 * par["mu"] * e[f] for f in ("txx", "tyy", "tzz")}
    rhs["txy"] = par["mxy"] * (dplus(g, s["vx"], Y) + dplus(g, s["vy"], X))
    rhs["txz"] = par["mxz"] * (dplus(g, s["vx"], Z) + dplus(g, s["vz"], X))
    rhs["tyz"] = par["myz"] * (dplus(g, s["vy"], Z) + dplus(g, s["vz"], Y))
    for f in ("txx", "tyy", "tzz", "txy", "txz", "tyz"):
        g.interior(s[f])[...] = ((1.0 - a) * g.interior(s[f]) + dt * rhs[f]) / (1.0 + a)


def zero_state(g: Grid):
    return {f: g.zeros() for f in FIELDS}


def forward(g: Grid, vp, vs, rho, src=None, q=None, rec=None, nt: int = 0, state=None):
    """nt updates.  Returns (state, d[nt][nr]): state maps each name in
    FIELDS to a padded array (v at step nt - 1/2, tau at step nt)."""
    assert g.ndim == 3
    s = zero_state(g) if state is None else {f: np.array(state[f], dtype=np.float64)
                                              for f in FIELDS}
    par = staggered_params(*medium(vp, vs, rho))
    a = 0.5 * g.dt * sponge_gamma(g)
    hinv = 1.0 / float(np.prod(g.spacing))
    ns = 0 if src is None else np.asarray(src).reshape(-1, 3).shape[0]
    nr = 0 if rec is None else np.asarray(rec).reshape(-1, 3).shape[0]
    if ns:
        snode, sw = sparse_weights(g, src)
    if nr:
        rnode, rw = sparse_weights(g, rec)
    d = np.zeros((nt, nr))
    for n in range(nt):
        for f in FIELDS[3:]:
            _fill(g, s[f], g.bc)
        velocity_update(g, s, par, a)
        for f in FIELDS[:3]:
            _fill(g, s[f], g.bc)
        stress_update(g, s, par, a)
        if ns:
            inj = np.zeros(g.padded_shape)
            np.add.at(inj.reshape(-1), snode.reshape(-1),
                      (sw * (hinv * np.asarray(q, dtype=np.float64)[n])[:, None]).reshape(-1))
            add = g.dt * g.interior(inj) / (1.0 + a)
            for f in ("txx", "tyy", "tzz"):
                g.interior(s[f])[...] += add
        if nr:
            tr = s["txx"] + s["tyy"] + s["tzz"]
            d[n] = (rw * tr.reshape(-1)[rnode]).sum(1)
    return s, d


def energy(g: Grid, v_old, v_new, tau, par):
    """Discrete energy of the undamped staggered scheme at step n:
    1/2 <v^(n+1/2), v^(n-1/2)>_{1/b} + 1/2 <tau^n, C^-1 tau^n>, with v_old,
    v_new the velocities at n -/+ 1/2 and tau the stresses at n (padded
    arrays keyed by FIELDS names).  C^-1 of the isotropic medium: strains
    (tau_ii - lambda tr(tau) / (3 lambda + 2 mu)) / (2 mu) and
    tau_ij / (2 mu_ij); each shear term counts twice in tau : eps."""
    I = g.interior
    e = 0.0
    for f, bname in (("vx", "bx"), ("vy", "by"), ("vz", "bz")):
        e += 0.5 * np.sum(I(v_new[f]) * I(v_old[f]) / par[bname])
    lam, mu = par["lam"], par["mu"]
    txx, tyy, tzz = I(tau["txx"]), I(tau["tyy"]), I(tau["tzz"])
    tr = txx + tyy + tzz
    e += np.sum((txx ** 2 + tyy ** 2 + tzz ** 2 - lam / (3.0 * lam + 2.0 * mu) * tr ** 2)
                / (4.0 * mu))
    for f, mname in (("txy", "mxy"), ("txz", "mxz"), ("tyz", "myz")):
        e += np.sum(I(tau[f]) ** 2 / (2.0 * par[mname]))
    return float(e)


def cfl_number(so: int) -> float:
    """sum_k |c_k|: with it the leapfrog is stable for
    vp dt sqrt(sum 1/h^2) * cfl_number <= 1 (the staggered derivative's
    symbol peaks at 2 sum |c_k| / h)."""
    return float(sum(abs(c) for c in staggered_weights_exact(so)))
