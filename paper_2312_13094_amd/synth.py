"""Seeded synthetic workloads for the finite-difference wave step.

This module only *generates inputs*: velocity models, anisotropy fields,
source signatures and acquisition geometry.  It contains none of the
scheme's arithmetic, and both the GPU path and the CPU oracle take their
inputs from here.

The paper evaluates on the Devito example models, which are not available
offline; the generators below stand in for them with the paper's shapes and
setup where it gives them (space order 8, a 40-point absorbing layer, a
Ricker source, hundreds of steps; problem-setup section).  Randomness uses
``numpy.random.default_rng(seed)`` in float64, rounded to float32 at the end.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

# Stability numbers S = -w_0 + 2 sum_k |w_k| of the centred second-derivative
# stencil of each space order (the largest magnitude of its Fourier symbol).
# Leapfrog is stable for v dt / h <= 2 / sqrt(ndim * S).  Used only to choose
# a time step for the synthetic workloads ("dt at 0.5 CFL").
_STAB = {2: 4.0, 4: 16.0 / 3.0, 8: 6.501587301587301, 12: 7.072943722943723,
         16: 7.426938775510204}


def courant_limit(so: int, ndim: int) -> float:
    return 2.0 / math.sqrt(ndim * _STAB[so])


def stable_dt(so: int, ndim: int, h: float, vmax: float, frac: float = 0.5) -> float:
    return frac * courant_limit(so, ndim) * h / vmax


def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet sampled at t_n = n dt, peak amplitude 1, delay t0 = 1/f0."""
    t0 = 1.0 / f0 if t0 is None else t0
    t = np.arange(nt) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def smooth_noise(shape, sigma: float, rng) -> np.ndarray:
    """N(0,1) noise smoothed by a periodic Gaussian filter of std `sigma` cells
    (applied in Fourier space), float64."""
    import scipy.fft as sfft
    x = rng.standard_normal(shape)
    workers = max(1, min(16, os.cpu_count() or 1))
    X = sfft.rfftn(x, workers=workers)
    del x
    for ax, n in enumerate(shape):
        k = np.fft.rfftfreq(n) if ax == len(shape) - 1 else np.fft.fftfreq(n)
        sh = [1] * len(shape)
        sh[ax] = -1
        X *= np.exp(-0.5 * (sigma * 2 * math.pi * k) ** 2).reshape(sh)
    return sfft.irfftn(X, s=shape, axes=list(range(len(shape))), workers=workers)


def minmax(a: np.ndarray, lo: float, hi: float) -> np.ndarray:
    a = (a - a.min()) / (a.max() - a.min())
    return lo + (hi - lo) * a


def layered_profile(nz: int, seed: int, vmin=1500.0, vmax=4500.0, min_thick=4) -> np.ndarray:
    """1-D velocity profile v(z) of 8-12 flat layers (fewer if nz is too
    short for them at min_thick cells each), velocities increasing with
    depth.  Thicknesses are min_thick plus a random composition of the
    remaining cells.  Returns float32 [nz]."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(8, 13))
    L = max(1, min(L, nz // min_thick))
    vel = np.sort(rng.uniform(vmin, vmax, L))
    spare = nz - L * min_thick
    bars = np.sort(rng.integers(0, spare + 1, L - 1))
    extra = np.diff(np.concatenate([[0], bars, [spare]]))
    edges = np.concatenate([[0], np.cumsum(min_thick + extra)])
    prof = np.empty(nz)
    for i in range(L):
        prof[edges[i]:edges[i + 1]] = vel[i]
    return prof.astype(np.float32)


def smooth_state(shape, seed: int, sigma: float = 4.0) -> np.ndarray:
    """A smooth random wavefield (unit std) for one-step parity checks."""
    rng = np.random.default_rng(seed)
    a = smooth_noise(tuple(shape), sigma, rng)
    return (a / a.std()).astype(np.float32)


@dataclass
class Acoustic:
    """One acoustic workload: DOMAIN shape (z,[y,]x), spacing, space order,
    sponge width, time step, steps, velocity, sources, receivers."""
    name: str
    shape: tuple
    spacing: tuple
    so: int
    nbl: int
    dt: float
    nt: int
    vmax: float
    boundary: int                       # 0 zero halo, 1 loopback (periodic)
    src: np.ndarray                     # [ns][ndim] metres from DOMAIN index 0
    rec: np.ndarray                     # [nr][ndim]
    q: np.ndarray                       # [nt][ns] float32
    vel_profile: np.ndarray | None = None   # [nz] when the model is flat in x, y
    vel: np.ndarray | None = field(default=None, repr=False)

    @property
    def ndim(self):
        return len(self.shape)

    def velocity(self) -> np.ndarray:
        """DOMAIN-shaped float32 velocity (materialised on demand)."""
        if self.vel is not None:
            return self.vel
        p = self.vel_profile.reshape((-1,) + (1,) * (self.ndim - 1))
        return np.ascontiguousarray(np.broadcast_to(p, self.shape)).astype(np.float32)

    @property
    def points(self) -> int:
        return int(np.prod(self.shape))


def cfg_2d(nt: int = 200) -> Acoustic:
    """2-D homogeneous acoustic: 128 x 128 physical grid + 20-point sponge per
    side (DOMAIN 168 x 168), h = 10 m, v = 1500 m/s, so 4, dt at 0.5 CFL,
    10 Hz Ricker at the centre, 128 receivers 20 m below the top of the
    physical region."""
    n, nbl, h, v, so = 168, 20, 10.0, 1500.0, 4
    dt = stable_dt(so, 2, h, v)
    c = (n - 1) / 2.0 * h
    src = np.array([[c, c]])
    rec = np.array([[(nbl + 2) * h, (nbl + i) * h] for i in range(128)])
    q = ricker(nt, dt, 10.0)[:, None]
    return Acoustic("acoustic2d_168sq_so4", (n, n), (h, h), so, nbl, dt, nt, v, 0,
                    src, rec, q, vel=np.full((n, n), v, dtype=np.float32))


def cfg_3d_layered(n: int = 512, nt: int = 500, seed: int = 2, so: int = 8, nbl: int = 40,
                   nrec: int | None = None) -> Acoustic:
    """3-D layered acoustic on an n^3 DOMAIN (headline: n = 512, so 8, 500 steps):
    seeded 8-12 flat layers, 1.5-4.5 km/s increasing with depth, 40-point
    sponge, 15 Hz Ricker, h = 10 m, dt at 0.5 CFL, a line of receivers, and
    loopback halo exchange of all six faces every step."""
    h = 10.0
    prof = layered_profile(n, seed)
    vmax = 4500.0
    dt = stable_dt(so, 3, h, vmax)
    s = n / 512.0
    src = np.array([[(50.5 * s) * h, (n / 2 - 0.5) * h, (n / 2 - 0.5) * h]])
    nr = n if nrec is None else nrec
    rz = round(45 * s)
    rec = np.array([[rz * h, (n / 2 - 0.5) * h, (i * (n - 1) / max(nr - 1, 1)) * h]
                    for i in range(nr)])
    q = ricker(nt, dt, 15.0)[:, None]
    return Acoustic("acoustic3d_%dcube_so%d_layered" % (n, so), (n, n, n), (h, h, h), so, nbl,
                    dt, nt, vmax, 1, src, rec, q, vel_profile=prof)


# First-derivative symbol peaks S1 = max_xi (2 sum_k a_k sin k xi)^2 of the
# centred first-derivative stencils; the rotated TTI operators are products
# of two first derivatives, stable for v sqrt(1+2 eps) dt sqrt(3 S1) / h <= 2.
_STAB1 = {4: 1.8830, 8: 2.9950, 12: 3.6897}


def tti_stable_dt(so: int, h: float, vmax: float, eps_max: float, frac: float = 0.5) -> float:
    return frac * 2.0 * h / (vmax * math.sqrt(1.0 + 2.0 * eps_max) * math.sqrt(3.0 * _STAB1[so]))


@dataclass
class TTI:
    """Pseudo-acoustic TTI workload: velocity, epsilon, delta, tilt theta and
    azimuth phi fields, plus acquisition (source at the centre)."""
    name: str
    shape: tuple
    spacing: tuple
    so: int
    nbl: int
    dt: float
    nt: int
    vmax: float
    eps_max: float
    src: np.ndarray
    rec: np.ndarray
    q: np.ndarray
    fields: dict = field(default=None, repr=False)   # v, eps, delta, theta, phi (float32)

    @property
    def points(self):
        return int(np.prod(self.shape))


def cfg_tti(n: int = 384, nt: int = 500, seed: int = 3, so: int = 12, nbl: int = 40) -> TTI:
    """3-D TTI on an n^3 DOMAIN (headline n = 384, so 12, 500 steps): v, eps,
    delta, theta, phi from Gaussian-filtered noise (sigma 8 cells, periodic)
    min-max mapped to [1500, 4500] m/s, [0, 0.3], [0, 0.15], [0, pi/4],
    [0, pi/4]; 40-point sponge, 20 Hz Ricker at the centre, h = 10 m."""
    h = 10.0
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    ranges = [("v", 1500.0, 4500.0), ("eps", 0.0, 0.3), ("delta", 0.0, 0.15),
              ("theta", 0.0, math.pi / 4), ("phi", 0.0, math.pi / 4)]
    f = {}
    for name, lo, hi in ranges:
        f[name] = minmax(smooth_noise(shape, 8.0, rng), lo, hi).astype(np.float32)
    vmax, eps_max = 4500.0, 0.3
    dt = tti_stable_dt(so, h, vmax, eps_max)
    c = (n / 2 - 0.5) * h
    src = np.array([[c, c, c]])
    s = n / 512.0
    rz = round(45 * s)
    rec = np.array([[rz * h, c, (i * (n - 1) / max(n - 1, 1)) * h] for i in range(n)])
    q = ricker(nt, dt, 20.0)[:, None]
    return TTI("tti3d_%dcube_so%d" % (n, so), shape, (h, h, h), so, nbl, dt, nt, vmax, eps_max,
               src, rec, q, fields=f)


# Sums sum_k |c_k| of the staggered first-derivative weights of each space
# order; the velocity-stress leapfrog is stable for
# vp dt sqrt(sum 1/h^2) sum_k |c_k| <= 1.  Used only to choose a time step.
_STAG = {2: 1.0, 4: 7.0 / 6.0, 8: 1.286309523809524, 12: 1.3390636273448773,
         16: 1.3703812355179543}


def elastic_stable_dt(so: int, h: float, vmax: float, frac: float = 0.5) -> float:
    return frac * h / (vmax * math.sqrt(3.0) * _STAG[so])


@dataclass
class Elastic:
    """Isotropic elastic workload: P and S velocities and density per node,
    an explosive source and receivers (they record the trace of the stress)."""
    name: str
    shape: tuple
    spacing: tuple
    so: int
    nbl: int
    dt: float
    nt: int
    vmax: float
    boundary: int
    src: np.ndarray
    rec: np.ndarray
    q: np.ndarray
    vp_profile: np.ndarray              # [nz]: the model is flat in x, y
    vs_profile: np.ndarray
    rho_profile: np.ndarray

    @property
    def points(self):
        return int(np.prod(self.shape))

    def fields(self):
        """DOMAIN-shaped float32 (vp, vs, rho)."""
        out = []
        for p in (self.vp_profile, self.vs_profile, self.rho_profile):
            out.append(np.ascontiguousarray(
                np.broadcast_to(p.reshape(-1, 1, 1), self.shape)).astype(np.float32))
        return tuple(out)


def cfg_elastic(n: int = 512, nt: int = 363, seed: int = 4, so: int = 8, nbl: int = 40,
                boundary: int = 1) -> Elastic:
    """3-D layered isotropic elastic on an n^3 DOMAIN (benchmark: 512^3, so 8,
    363 steps, the paper's elastic step count for 512 ms): vp from the seeded layered profile (1.5-4.5 km/s), vs = vp /
    sqrt(3) (a Poisson solid), rho = 310 vp^0.25 kg/m^3 (Gardner's relation);
    40-point sponge, 15 Hz Ricker explosive source near the top, a line of
    receivers, h = 10 m, dt at 0.5 CFL, loopback halos for all nine
    components."""
    h = 10.0
    vp = layered_profile(n, seed).astype(np.float64)
    vs = vp / math.sqrt(3.0)
    rho = 310.0 * vp ** 0.25
    vmax = 4500.0
    dt = elastic_stable_dt(so, h, vmax)
    s = n / 512.0
    c = (n / 2 - 0.5) * h
    src = np.array([[(50.5 * s) * h, c, c]])
    rz = round(45 * s)
    rec = np.array([[rz * h, c, (i * (n - 1) / max(n - 1, 1)) * h] for i in range(n)])
    q = ricker(nt, dt, 15.0)[:, None]
    return Elastic("elastic3d_%dcube_so%d_layered" % (n, so), (n, n, n), (h, h, h), so, nbl, dt,
                   nt, vmax, boundary, src, rec, q, vp.astype(np.float32),
                   vs.astype(np.float32), rho.astype(np.float32))


def sls_times(q, f0):
    """(tau_e, tau_s) of one standard linear solid whose quality factor
    peaks at q at frequency f0 (Blanch et al. 1995): w0 = 2 pi f0,
    tau_s = (sqrt(1 + 1/q^2) - 1/q) / w0, tau_e = 1 / (w0^2 tau_s)."""
    w0 = 2.0 * math.pi * f0
    ts = (np.sqrt(1.0 + 1.0 / (q * q)) - 1.0 / q) / w0
    return 1.0 / (w0 * w0 * ts), ts


@dataclass
class Visco(Elastic):
    """Visco-elastic workload: the elastic one plus the relaxation times
    (tau_ep, tau_es, tau_s) per depth."""
    tep_profile: np.ndarray = None
    tes_profile: np.ndarray = None
    ts_profile: np.ndarray = None

    def fields(self):
        """DOMAIN-shaped float32 (vp, vs, rho, tau_ep, tau_es, tau_s)."""
        out = []
        for p in (self.vp_profile, self.vs_profile, self.rho_profile, self.tep_profile,
                  self.tes_profile, self.ts_profile):
            out.append(np.ascontiguousarray(
                np.broadcast_to(p.reshape(-1, 1, 1), self.shape)).astype(np.float32))
        return tuple(out)

    def profiles(self):
        return (self.vp_profile, self.vs_profile, self.rho_profile, self.tep_profile,
                self.tes_profile, self.ts_profile)


def cfg_visco(n: int = 512, nt: int = 251, seed: int = 4, so: int = 8, nbl: int = 40,
              boundary: int = 1, f0: float = 15.0) -> Visco:
    """3-D layered visco-elastic on an n^3 DOMAIN (benchmark: 512^3, so 8,
    251 steps, the paper's visco-elastic step count for 512 ms): the elastic
    workload's vp, vs, rho with quality factors Qp = 40 vp / 1 km/s and
    Qs = Qp / 2 (stiffer layers attenuate less), one relaxation mechanism
    centred on the 15 Hz source frequency."""
    e = cfg_elastic(n=n, nt=nt, seed=seed, so=so, nbl=nbl, boundary=boundary)
    vp = e.vp_profile.astype(np.float64)
    qp = 40.0 * vp / 1000.0
    qs = qp / 2.0
    tep, ts = sls_times(qp, f0)
    # one stress relaxation time per node (the P mechanism's); the S strain
    # relaxation time then solves Qs(w0) = (1 + w0^2 tes ts) / (w0 (tes - ts)) = qs
    w0 = 2.0 * math.pi * f0
    tes = (qs * w0 * ts + 1.0) / (w0 * (qs - w0 * ts))
    vmax = float(np.max(vp * np.sqrt(tep / ts))) * 1.001
    dt = elastic_stable_dt(so, e.spacing[0], vmax)
    q = ricker(nt, dt, f0)[:, None]
    return Visco("visco3d_%dcube_so%d_layered" % (n, so), e.shape, e.spacing, so, nbl, dt, nt,
                 vmax, boundary, e.src, e.rec, q, e.vp_profile, e.vs_profile, e.rho_profile,
                 tep.astype(np.float32), tes.astype(np.float32), ts.astype(np.float32))


@dataclass
class FWIBatch:
    """Batched-gradient workload: a full model (layered + Gaussian anomaly),
    its layered starting model, and per-shot apertures with acquisition."""
    name: str
    full_shape: tuple
    spacing: tuple
    so: int
    nbl: int
    dt: float
    nt: int
    ckpt_every: int
    vmax: float
    shapes: list
    origins: list
    src: list          # per shot [1][3] metres in aperture coordinates
    rec: list          # per shot [nr][3]
    q: np.ndarray      # [nt][1]
    profile: np.ndarray = field(default=None, repr=False)
    anomaly: tuple = (0.6, 0.5, 0.5, 12.0, 300.0)   # centre fractions (z,y,x), sigma cells, dv

    def true_velocity(self) -> np.ndarray:
        v = self.start_velocity().astype(np.float64)
        fz, fy, fx, sig, dv = self.anomaly
        nz, ny, nx = self.full_shape
        z = (np.arange(nz) - fz * nz)[:, None, None]
        y = (np.arange(ny) - fy * ny)[None, :, None]
        x = (np.arange(nx) - fx * nx)[None, None, :]
        v += dv * np.exp(-(z * z + y * y + x * x) / (2 * sig * sig))
        return np.minimum(v, self.vmax).astype(np.float32)

    def start_velocity(self) -> np.ndarray:
        p = self.profile.reshape(-1, 1, 1)
        return np.ascontiguousarray(np.broadcast_to(p, self.full_shape)).astype(np.float32)


def cfg_fwi_batch(n: int = 512, nshots: int = 16, side_lo: int = 24, side_hi: int = 40,
                  unit: int = 8, nt: int = 800, ckpt_every: int = 50, seed: int = 4,
                  so: int = 8, nbl: int = 40, sigma: float = 12.0) -> FWIBatch:
    """16 shots (seeds 4000+i) with cube apertures of side unit * U{side_lo..side_hi}
    (192..320 at the defaults), placed uniformly inside an n^3 layered model
    (seed 4) with a +300 m/s Gaussian anomaly (sigma 12 cells) at
    (0.6 nz, ny/2, nx/2); source 44 cells deep at the aperture centre,
    receivers 42 cells deep along x; so 8, 800 steps, checkpoint every 50."""
    h = 10.0
    prof = layered_profile(n, seed)
    vmax = 4500.0
    dt = stable_dt(so, 3, h, vmax)
    shapes, origins, srcs, recs = [], [], [], []
    for i in range(nshots):
        rng = np.random.default_rng(4000 + i)
        s = unit * int(rng.integers(side_lo, side_hi + 1))
        s = min(s, n)
        o = [int(rng.integers(0, n - s + 1)) for _ in range(3)]
        shapes.append((s, s, s))
        origins.append(tuple(o))
        zs = min(44, s - 2)
        zr = min(42, s - 2)
        c = (s // 2) * h
        srcs.append(np.array([[zs * h, c, c]]))
        recs.append(np.array([[zr * h, c, x * h] for x in range(s)]))
    q = ricker(nt, dt, 15.0)[:, None]
    return FWIBatch("fwi_batch_%dshots_%dcube" % (nshots, n), (n, n, n), (h, h, h), so, nbl, dt,
                    nt, ckpt_every, vmax, shapes, origins, srcs, recs, q, profile=prof,
                    anomaly=(0.6, 0.5, 0.5, sigma, 300.0))


@dataclass
class Learned:
    """Learned-correction workload: a fine high-order grid and a 2x coarser
    low-order grid over the same region, with models, source and receivers
    on coarse nodes (which are also fine nodes)."""
    name: str
    n_fine: int
    h_fine: float
    so_fine: int
    so_coarse: int
    nbl_fine: int
    dt_fine: float
    nt_fine: int
    vmax: float
    src_idx: tuple          # fine-grid index of the source (even)
    rec_z: int              # fine-grid depth index of the receiver line (even)
    rec_y: int              # fine-grid crossline index of the receiver line (even)
    f0: float
    train_seeds: list
    test_seeds: list

    @property
    def n_coarse(self):
        return self.n_fine // 2

    @property
    def h_coarse(self):
        return 2 * self.h_fine

    @property
    def dt_coarse(self):
        return 2 * self.dt_fine

    @property
    def nt_coarse(self):
        return self.nt_fine // 2

    @property
    def nbl_coarse(self):
        return self.nbl_fine // 2

    def velocity(self, seed: int) -> np.ndarray:
        """Fine-grid model: layered (8-12 layers) plus 0-3 Gaussian anomalies of
        +-10-20 %, sigma 8-24 fine cells, clipped to [1500, 4500] m/s."""
        n = self.n_fine
        v = np.broadcast_to(layered_profile(n, seed).reshape(-1, 1, 1), (n, n, n)).astype(np.float64)
        rng = np.random.default_rng(seed + 100000)
        k = int(rng.integers(0, 4))
        zz = np.arange(n)[:, None, None]
        yy = np.arange(n)[None, :, None]
        xx = np.arange(n)[None, None, :]
        for _ in range(k):
            c = rng.uniform(0.2 * n, 0.8 * n, 3)
            sig = rng.uniform(8, 24) * n / 256.0
            amp = rng.uniform(0.10, 0.20) * rng.choice([-1.0, 1.0])
            g = np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) / (2 * sig * sig))
            v = v * (1.0 + amp * g)
        return np.clip(v, 1500.0, 4500.0).astype(np.float32)

    def src_fine(self):
        return np.array([[i * self.h_fine for i in self.src_idx]])

    def rec_fine(self):
        n = self.n_fine
        return np.array([[self.rec_z * self.h_fine, self.rec_y * self.h_fine, 2 * i * self.h_fine]
                         for i in range(n // 2)])

    def q_fine(self):
        return ricker(self.nt_fine, self.dt_fine, self.f0)[:, None]

    def q_coarse(self):
        return ricker(self.nt_coarse, self.dt_coarse, self.f0)[:, None]


def cfg_learned(n_fine: int = 256, nt_fine: int = 1000, ntrain: int = 64, ntest: int = 8) -> Learned:
    """Fine 256^3 (h = 10 m, so 8, 40-point layer, dt at 0.5 CFL) and coarse
    128^3 (h = 20 m, so 4, 20-point layer, 2 dt); 1000 fine / 500 coarse
    steps; 15 Hz Ricker near the top centre; 128 receivers on coarse nodes
    near the top, on an inline offset n/4 crossline from the source (the
    nearest receiver is 640 m away at n = 256, beyond the source's near
    field); training seeds 5000.., held-out seeds 5100.."""
    h = 10.0
    vmax = 4500.0
    dt = stable_dt(8, 3, h, vmax)
    s = n_fine / 256.0
    src = (2 * round(24 * s), n_fine // 2, n_fine // 2)
    return Learned("learned_%dfine_%dcoarse" % (n_fine, n_fine // 2), n_fine, h, 8, 4,
                   2 * round(20 * s), dt, nt_fine, vmax, src, 2 * round(26 * s),
                   n_fine // 2 + 2 * round(n_fine / 8), 15.0,
                   list(range(5000, 5000 + ntrain)), list(range(5100, 5100 + ntest)))
