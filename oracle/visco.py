"""FP64 oracle of the visco-elastic velocity-stress step with one relaxation
mechanism (test infrastructure only: tests, smoke() and bench.py's CPU
baseline use it; the HIP path never does).

Paper, appendix "Visco-elastic", equations (model-equations) and the table
of their parameters: relaxed moduli pi (P, the analogue of lambda + 2 mu)
and mu (S), strain relaxation times tau_ep, tau_es and the stress
relaxation time tau_s, one memory variable r_ij per stress component.  The
paper prints the memory-variable forcing with the ratios tau_e / tau_s; the
reading used here carries (tau_e / tau_s - 1) there, so that tau_e = tau_s
(no attenuation) leaves the memory variables at rest and the system reduces
to the elastic one (the form of Robertson et al. 1994, which the paper
cites):

    v_t    = b div(sigma)
    s_ii_t = P_u tr(e) + 2 M_u (e_ii - tr(e)) + r_ii
    s_ij_t = M_u (e_ij + e_ji) + r_ij                              (i != j)
    r_ii_t = -(r_ii + P_d tr(e) + 2 M_d (e_ii - tr(e))) / tau_s
    r_ij_t = -(r_ij + M_d (e_ij + e_ji)) / tau_s
    with e_ij = d_i v_j, P_u = pi tau_ep / tau_s, M_u = mu tau_es / tau_s,
    P_d = pi (tau_ep / tau_s - 1), M_d = mu (tau_es / tau_s - 1).

Discretisation (first order in time, as the paper states for this model):
the staggered grid, staggered derivatives, velocity update, damping, source
and receivers of the elastic oracle (oracle/elastic.py); then per update
    r^(n+1)   = r^n - (dt / tau_s) (r^n + forcing(e(v^(n+1/2))))   (explicit Euler,
                no damping: the memory variables relax on their own)
    sigma^(n+1) = [(1 - a) sigma^n + dt (unrelaxed(e) + r^(n+1))] / (1 + a).
Each r_ij sits at its sigma_ij position.  At a shear-stress position the
coefficients M_u, M_d and 1/tau_s are the means over the four nodes of its
staggered plane (node values beyond DOMAIN repeat the last one); the normal
stresses use node values.
"""
from __future__ import annotations

import numpy as np

from . import Grid, sparse_weights, sponge_gamma
from .elastic import X, Y, Z, _next, dminus, dplus, velocity_update
from .tti import _fill

FIELDS = ("vx", "vy", "vz", "txx", "tyy", "tzz", "txy", "txz", "tyz",
          "rxx", "ryy", "rzz", "rxy", "rxz", "ryz")


def _mean4(m, p, q):
    return 0.25 * (m + _next(m, p) + _next(m, q) + _next(_next(m, p), q))


def coefficients(vp, vs, rho, tau_ep, tau_es, tau_s):
    """Per-position coefficients (DOMAIN arrays): bx, by, bz (buoyancy at
    the velocities), and for each stress position the unrelaxed moduli
    (pu, mu at nodes; mu_xy ...), the memory forcing moduli (pd, md; md_xy
    ...) and the inverse stress relaxation time (ks; ks_xy ...)."""
    vp, vs, rho, tep, tes, ts = (np.asarray(a, dtype=np.float64)
                                 for a in (vp, vs, rho, tau_ep, tau_es, tau_s))
    b = 1.0 / rho
    pi, mu = rho * vp * vp, rho * vs * vs
    c = {"bx": 0.5 * (b + _next(b, X)), "by": 0.5 * (b + _next(b, Y)),
         "bz": 0.5 * (b + _next(b, Z)),
         "pu": pi * tep / ts, "mu": mu * tes / ts,
         "pd": pi * (tep / ts - 1.0), "md": mu * (tes / ts - 1.0), "ks": 1.0 / ts}
    for sfx, (p, q) in (("xy", (Y, X)), ("xz", (Z, X)), ("yz", (Z, Y))):
        c["mu_" + sfx] = _mean4(c["mu"], p, q)
        c["md_" + sfx] = _mean4(c["md"], p, q)
        c["ks_" + sfx] = _mean4(c["ks"], p, q)
    return c


def stress_memory_update(g: Grid, s, c, a):
    """r^(n+1) and sigma^(n+1) from r^n, sigma^n and v^(n+1/2) (halos of v
    filled)."""
    dt = g.dt
    I = g.interior
    e = {"xx": dminus(g, s["vx"], X), "yy": dminus(g, s["vy"], Y), "zz": dminus(g, s["vz"], Z)}
    tr = e["xx"] + e["yy"] + e["zz"]
    sh = {"xy": dplus(g, s["vx"], Y) + dplus(g, s["vy"], X),
          "xz": dplus(g, s["vx"], Z) + dplus(g, s["vz"], X),
          "yz": dplus(g, s["vy"], Z) + dplus(g, s["vz"], Y)}
    for ii in ("xx", "yy", "zz"):
        dev = e[ii] - tr
        r = I(s["r" + ii])
        r[...] = r - dt * c["ks"] * (r + c["pd"] * tr + 2.0 * c["md"] * dev)
        t = I(s["t" + ii])
        t[...] = ((1.0 - a) * t + dt * (c["pu"] * tr + 2.0 * c["mu"] * dev + r)) / (1.0 + a)
    for ij in ("xy", "xz", "yz"):
        r = I(s["r" + ij])
        r[...] = r - dt * c["ks_" + ij] * (r + c["md_" + ij] * sh[ij])
        t = I(s["t" + ij])
        t[...] = ((1.0 - a) * t + dt * (c["mu_" + ij] * sh[ij] + r)) / (1.0 + a)


def zero_state(g: Grid):
    return {f: g.zeros() for f in FIELDS}


def forward(g: Grid, vp, vs, rho, tau_ep, tau_es, tau_s, src=None, q=None, rec=None,
            nt: int = 0, state=None):
    """nt updates.  Returns (state, d[nt][nr]) with state keyed by FIELDS
    (padded arrays: v at step nt - 1/2, sigma and r at step nt)."""
    assert g.ndim == 3
    s = zero_state(g) if state is None else {f: np.array(state[f], dtype=np.float64)
                                              for f in FIELDS}
    c = coefficients(vp, vs, rho, tau_ep, tau_es, tau_s)
    par = {"bx": c["bx"], "by": c["by"], "bz": c["bz"]}
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
        for f in FIELDS[3:9]:
            _fill(g, s[f], g.bc)
        velocity_update(g, s, par, a)
        for f in FIELDS[:3]:
            _fill(g, s[f], g.bc)
        stress_memory_update(g, s, c, a)
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


def sls_relaxation_times(q, f0):
    """Relaxation times (tau_e, tau_s) of one standard linear solid whose
    quality factor peaks at Q = q at frequency f0: tau_s = (sqrt(1 + 1/q^2)
    - 1/q) / w0, tau_e = 1 / (w0^2 tau_s), w0 = 2 pi f0 (Blanch et al.
    1995).  Used by tests to build media with a prescribed Q."""
    w0 = 2.0 * np.pi * f0
    ts = (np.sqrt(1.0 + 1.0 / (q * q)) - 1.0 / q) / w0
    return 1.0 / (w0 * w0 * ts), ts
