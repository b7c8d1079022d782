"""FP64 oracle of the pseudo-acoustic TTI step (test infrastructure only).

Paper, appendix "Anisotropic acoustic (TTI)", equation (rot): the rotated
second derivative G_xbar_xbar = D_xbar^T D_xbar with
D_xbar = cos(theta)cos(phi) d/dx + cos(theta)sin(phi) d/dy - sin(theta) d/dz;
the full coupled system is not printed, the paper defers it to its
references (Zhang et al. 2011; Louboutin et al. 2018).  The reading used
here is their two-field form:

    p_tt = v^2 [ (1 + 2 eps) H_xy p + sqrt(1 + 2 delta) H_z r ]
    r_tt = v^2 [ sqrt(1 + 2 delta) H_xy p + H_z r ]

with the tilted symmetry axis a = (sin t cos f, sin t sin f, cos t) (x, y, z
components; t = theta the tilt from vertical, f = phi the azimuth; a is the
unit vector orthogonal to the printed xbar direction), and

    H_z  u = div_h( a (a . grad_h u) )          = -D_zbar^T D_zbar u
    H_xy u = div_h( (I - a a^T) grad_h u )      = -(D_xbar^T D_xbar + D_ybar^T D_ybar) u

where grad_h / div_h use centred first-derivative weights of order so.
The intermediate vectors (I - a a^T) grad p and a (a . grad r) are formed on
DOMAIN and extended by zero outside it (bc 0; then D^T is an exact
transpose), or periodically (bc 1, used only by the exact plane-wave pin).
Damping, source injection into both fields and the time alignment follow the
acoustic scheme; receivers record p.

Arrays are (z, y, x); padded fields carry a halo of r = so/2.
"""
from __future__ import annotations

import math

import numpy as np

from . import Grid, d1_weights, sparse_weights, sponge_gamma


def axis_vector(theta, phi):
    """Symmetry axis a as (a_z, a_y, a_x) arrays (our axis order)."""
    return (np.cos(theta), np.sin(theta) * np.sin(phi), np.sin(theta) * np.cos(phi))


def _fill(g: Grid, u: np.ndarray, bc: int) -> None:
    """Halo of a padded array: zero (bc 0) or periodic (bc 1)."""
    r = g.r
    n = g.shape
    if bc == 0:
        inner = g.interior(u).copy()
        u[...] = 0.0
        g.interior(u)[...] = inner
        return
    for ax in range(3):
        sl_lo = [slice(r, r + s) for s in n]
        sl_hi = [slice(r, r + s) for s in n]
        src_lo = [slice(r, r + s) for s in n]
        src_hi = [slice(r, r + s) for s in n]
        sl_lo[ax] = slice(0, r)
        src_lo[ax] = slice(n[ax], n[ax] + r)
        sl_hi[ax] = slice(n[ax] + r, n[ax] + 2 * r)
        src_hi[ax] = slice(r, 2 * r)
        u[tuple(sl_lo)] = u[tuple(src_lo)]
        u[tuple(sl_hi)] = u[tuple(src_hi)]


def d1(g: Grid, u: np.ndarray, axis: int, h: float) -> np.ndarray:
    """Centred first derivative along `axis` on DOMAIN from a padded array:
    sum_k a_k (u[i+k] - u[i-k]) / h."""
    r = g.r
    a = d1_weights(g.so)
    n = g.shape
    out = np.zeros(n)
    base = [slice(r, r + s) for s in n]
    for k in range(1, r + 1):
        plus = list(base)
        minus = list(base)
        plus[axis] = slice(r + k, r + k + n[axis])
        minus[axis] = slice(r - k, r - k + n[axis])
        out += a[k - 1] * (u[tuple(plus)] - u[tuple(minus)])
    return out / h


def grad(g: Grid, u: np.ndarray):
    return [d1(g, u, ax, g.spacing[ax]) for ax in range(3)]


def div(g: Grid, w, bc: int) -> np.ndarray:
    """sum_i d_i w_i with each DOMAIN-shaped w_i extended by zero (bc 0) or
    periodically (bc 1)."""
    out = np.zeros(g.shape)
    for ax in range(3):
        wp = g.pad(w[ax])
        _fill(g, wp, bc)
        out += d1(g, wp, ax, g.spacing[ax])
    return out


def operators(g: Grid, p: np.ndarray, r: np.ndarray, theta, phi, bc: int):
    """(H_xy p, H_z r) on DOMAIN; p, r padded with their halo filled."""
    az, ay, ax = axis_vector(theta, phi)
    a = (az, ay, ax)
    gp = grad(g, p)
    gr = grad(g, r)
    ap = az * gp[0] + ay * gp[1] + ax * gp[2]
    ar = az * gr[0] + ay * gr[1] + ax * gr[2]
    w = [gp[i] - a[i] * ap for i in range(3)]     # (I - a a^T) grad p
    s = [a[i] * ar for i in range(3)]             # a (a . grad r)
    return div(g, w, bc), div(g, s, bc)


def forward(g: Grid, v, eps, delta, theta, phi, src=None, q=None, rec=None, nt=0,
            p0=None, pm=None, r0=None, rm=None, gamma=None):
    """nt leapfrog updates of the TTI system.  Returns
    (p^nt, p^(nt-1), r^nt, r^(nt-1), d[nt][nr]) with padded fields.  gamma,
    if given, is the DOMAIN-shaped damping rate to use instead of g's own
    layer (a window of a larger grid keeps that grid's damping)."""
    bc = g.bc
    v = np.asarray(v, dtype=np.float64)
    p = g.zeros() if p0 is None else np.array(p0, dtype=np.float64)
    po = g.zeros() if pm is None else np.array(pm, dtype=np.float64)
    r = g.zeros() if r0 is None else np.array(r0, dtype=np.float64)
    ro = g.zeros() if rm is None else np.array(rm, dtype=np.float64)
    gam = sponge_gamma(g) if gamma is None else np.asarray(gamma, dtype=np.float64)
    a = 0.5 * g.dt * gam
    c = v * v * g.dt * g.dt
    c_pp = c * (1.0 + 2.0 * np.asarray(eps, dtype=np.float64))
    c_x = c * np.sqrt(1.0 + 2.0 * np.asarray(delta, dtype=np.float64))
    hinv = 1.0 / float(np.prod(g.spacing))
    ns = 0 if src is None else np.asarray(src).reshape(-1, 3).shape[0]
    nr = 0 if rec is None else np.asarray(rec).reshape(-1, 3).shape[0]
    if ns:
        snode, sw = sparse_weights(g, src)
    if nr:
        rnode, rw = sparse_weights(g, rec)
    d = np.zeros((nt, nr))
    for n in range(nt):
        _fill(g, p, bc)
        _fill(g, r, bc)
        hxy, hz = operators(g, p, r, theta, phi, bc)
        f = np.zeros(g.padded_shape)
        if ns:
            np.add.at(f.reshape(-1), snode.reshape(-1),
                      (sw * (hinv * np.asarray(q, dtype=np.float64)[n])[:, None]).reshape(-1))
        f = g.interior(f)
        pn = (2.0 * g.interior(p) - (1.0 - a) * g.interior(po) +
              c_pp * hxy + c_x * hz + c * f) / (1.0 + a)
        rn = (2.0 * g.interior(r) - (1.0 - a) * g.interior(ro) +
              c_x * hxy + c * hz + c * f) / (1.0 + a)
        po, ro = p, r
        p, r = g.pad(pn), g.pad(rn)
        if nr:
            d[n] = (rw * p.reshape(-1)[rnode]).sum(1)
    return p, po, r, ro, d


def stability_number(so: int) -> float:
    """max over xi of (2 sum_k a_k sin(k xi))^2: the squared peak of the
    first-derivative symbol (on a fine sampling of xi)."""
    a = d1_weights(so)
    xi = np.linspace(0.0, math.pi, 20001)
    sym = 2.0 * sum(a[k - 1] * np.sin(k * xi) for k in range(1, len(a) + 1))
    return float((sym ** 2).max())
