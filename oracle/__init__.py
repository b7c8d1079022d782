"""Plain FP64 CPU oracle for the explicit finite-difference wave step.

TEST INFRASTRUCTURE ONLY.  This package is the checker the GPU library is
compared against; only the tests, the smoke check and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library: the
arithmetic lives in ``fd_oracle.c`` (acoustic forward/adjoint/gradient, halo
faces, sparse weights), ``tti.py`` (pseudo-acoustic TTI) and ``nn.py``
(the learned-correction network), each citing the passage it follows.

The C part is built with gcc on first use (or by ``__graft_entry__.build``)
into ``oracle/_fd_oracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd_oracle.c")
_SO = os.path.join(_HERE, "_fd_oracle.so")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _OrGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double * 3),
                ("so", ctypes.c_int), ("nbl", ctypes.c_int), ("dt", ctypes.c_double),
                ("vmax", ctypes.c_double), ("bc", ctypes.c_int)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        g = P(_OrGrid)
        dp = P(ctypes.c_double)
        i64p = P(ctypes.c_int64)
        lib.or_field_elems.argtypes = [g]; lib.or_field_elems.restype = ctypes.c_int64
        lib.or_index.argtypes = [g, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.or_index.restype = ctypes.c_int64
        lib.or_d2_weights.argtypes = [ctypes.c_int, dp]
        lib.or_d1_weights.argtypes = [ctypes.c_int, dp]
        lib.or_sponge_gamma.argtypes = [g, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.or_sponge_gamma.restype = ctypes.c_double
        lib.or_face_elems.argtypes = [g, ctypes.c_int]; lib.or_face_elems.restype = ctypes.c_int64
        lib.or_pack_face.argtypes = [g, dp, ctypes.c_int, dp]
        lib.or_unpack_face.argtypes = [g, dp, ctypes.c_int, dp]
        lib.or_fill_halo.argtypes = [g, dp]; lib.or_fill_halo.restype = None
        lib.or_laplacian.argtypes = [g, dp, dp]; lib.or_laplacian.restype = None
        lib.or_sparse_weights.argtypes = [g, dp, ctypes.c_int, i64p, dp]
        lib.or_forward.argtypes = [g, dp, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp,
                                   ctypes.c_int, dp]
        lib.or_adjoint.argtypes = [g, dp, dp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp,
                                   ctypes.c_int, dp, dp]
        lib.or_heat.argtypes = [g, dp, ctypes.c_int]; lib.or_heat.restype = None
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Grid description (DOMAIN shape in (z, y, x) order; 2-D grids are (z, x)).

    bc: 0 zero halo, 1 periodic halo realised by face pack/unpack, 2 halo left
    as the caller filled it (subdomain exchange)."""
    shape: tuple
    spacing: tuple
    so: int
    dt: float
    nbl: int = 0
    vmax: float = 0.0
    bc: int = 0
    _c: _OrGrid = field(default=None, repr=False)

    def __post_init__(self):
        self.ndim = len(self.shape)
        assert self.ndim in (2, 3)
        if self.ndim == 2:
            n = (self.shape[0], 1, self.shape[1])
            h = (self.spacing[0], 1.0, self.spacing[1])
        else:
            n, h = tuple(self.shape), tuple(self.spacing)
        self.n3, self.h3 = n, h
        c = _OrGrid()
        c.ndim = self.ndim
        for i in range(3):
            c.n[i] = int(n[i])
            c.h[i] = float(h[i])
        c.so, c.nbl, c.dt, c.vmax, c.bc = int(self.so), int(self.nbl), float(self.dt), \
            float(self.vmax), int(self.bc)
        self._c = c

    @property
    def r(self):
        return self.so // 2

    @property
    def padded_shape(self):
        r = self.r
        if self.ndim == 2:
            return (self.shape[0] + 2 * r, self.shape[1] + 2 * r)
        return tuple(s + 2 * r for s in self.shape)

    def zeros(self):
        return np.zeros(self.padded_shape, dtype=np.float64)

    def interior(self, a):
        """DOMAIN view of a padded array."""
        r = self.r
        return a[tuple(slice(r, r + s) for s in self.shape)]

    def pad(self, dom):
        """Padded copy of a DOMAIN-shaped array, halo zero."""
        out = self.zeros()
        self.interior(out)[...] = dom
        return out


def d2_weights(so: int) -> np.ndarray:
    w = np.zeros(so // 2 + 1)
    if _L().or_d2_weights(so, _dp(w)) != 0:
        raise ValueError("bad space order %r" % so)
    return w


def d1_weights(so: int) -> np.ndarray:
    a = np.zeros(so // 2)
    if _L().or_d1_weights(so, _dp(a)) != 0:
        raise ValueError("bad space order %r" % so)
    return a


def sponge_gamma(g: Grid) -> np.ndarray:
    """DOMAIN-shaped damping rate of the absorbing layer."""
    L = _L()
    nz, ny, nx = g.n3
    out = np.zeros((nz, ny, nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                out[z, y, x] = L.or_sponge_gamma(ctypes.byref(g._c), z, y, x)
    return out.reshape(g.shape)


def sponge_gamma_box(g: Grid, lo, hi) -> np.ndarray:
    """The damping rate of grid g on the box of DOMAIN indices [lo, hi) (one
    (z, y, x) triple each; 3-D grids), point by point as sponge_gamma: for a
    window of a larger grid whose own boundary is not the damping layer's."""
    return sponge_gamma_at(g, *(range(int(l), int(h)) for l, h in zip(lo, hi)))


def sponge_gamma_at(g: Grid, zs, ys, xs) -> np.ndarray:
    """The damping rate of grid g at every (z, y, x) of the three lists of
    DOMAIN indices (any order, repeats allowed), point by point as
    sponge_gamma: for a window that wraps round a periodic grid."""
    L = _L()
    zs, ys, xs = ([int(v) for v in a] for a in (zs, ys, xs))
    out = np.zeros((len(zs), len(ys), len(xs)))
    for i, z in enumerate(zs):
        for j, y in enumerate(ys):
            for k, x in enumerate(xs):
                out[i, j, k] = L.or_sponge_gamma(ctypes.byref(g._c), z, y, x)
    return out


def laplacian(g: Grid, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    lap = np.zeros(g.shape)
    _L().or_laplacian(ctypes.byref(g._c), _dp(u), _dp(lap))
    return lap


def fill_halo(g: Grid, u: np.ndarray) -> None:
    _L().or_fill_halo(ctypes.byref(g._c), _dp(u))


def face_elems(g: Grid, f: int) -> int:
    return int(_L().or_face_elems(ctypes.byref(g._c), f))


def pack_face(g: Grid, u: np.ndarray, f: int) -> np.ndarray:
    buf = np.zeros(max(face_elems(g, f), 1))
    if _L().or_pack_face(ctypes.byref(g._c), _dp(u), f, _dp(buf)) != 0:
        raise ValueError("bad face")
    return buf[:face_elems(g, f)]


def unpack_face(g: Grid, u: np.ndarray, f: int, buf: np.ndarray) -> None:
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    assert buf.size == face_elems(g, f)
    if buf.size == 0:
        return
    if _L().or_unpack_face(ctypes.byref(g._c), _dp(u), f, _dp(buf)) != 0:
        raise ValueError("bad face")


def sparse_weights(g: Grid, coords: np.ndarray):
    """(node padded linear indices, weights), each [npts][2^ndim]."""
    coords = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, g.ndim)
    n = coords.shape[0]
    nc = 1 << g.ndim
    node = np.zeros((max(n, 1), nc), dtype=np.int64)
    wt = np.zeros((max(n, 1), nc))
    rc = _L().or_sparse_weights(ctypes.byref(g._c), _dp(coords), n,
                                node.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(wt))
    if rc != 0:
        raise ValueError("sparse point outside the grid")
    return node[:n], wt[:n]


def _coords(g, c):
    if c is None:
        return np.zeros((0, g.ndim)), 0
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1, g.ndim)
    return c, c.shape[0]


def forward(g: Grid, v, src=None, q=None, rec=None, nt: int = 0, u0=None, um=None,
            history: bool = False):
    """nt leapfrog updates.  Returns (u^nt, u^(nt-1), d[nt][nr], hist|None).

    u0/um are padded initial states u^0, u^-1 (default zero)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == tuple(g.shape)
    u = g.zeros() if u0 is None else np.array(u0, dtype=np.float64, order="C")
    uo = g.zeros() if um is None else np.array(um, dtype=np.float64, order="C")
    src, ns = _coords(g, src)
    rec, nr = _coords(g, rec)
    qq = np.zeros((nt, ns)) if q is None else np.ascontiguousarray(q, dtype=np.float64)
    assert qq.shape == (nt, ns)
    d = np.zeros((nt, nr))
    hist = np.zeros((nt + 2,) + tuple(g.shape)) if history else None
    rc = _L().or_forward(ctypes.byref(g._c), _dp(v), _dp(u), _dp(uo), ns, _dp(src.copy()),
                         _dp(qq), nr, _dp(rec.copy()), _dp(d), nt, _dp(hist))
    if rc != 0:
        raise ValueError("sparse point outside the grid")
    return u, uo, d, hist


def adjoint(g: Grid, v, rec, resid, src=None, nt: int = 0, hist=None):
    """Transposed modelling.  Returns (lambda_0, lambda_1, qadj[nt][ns], grad_m|None).

    grad_m (dJ/dm for J = 1/2 |d - d_obs|^2 with resid = d - d_obs) is
    accumulated when the forward history is given."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    lam, lamo = g.zeros(), g.zeros()
    rec, nr = _coords(g, rec)
    src, ns = _coords(g, src)
    resid = np.ascontiguousarray(resid, dtype=np.float64)
    assert resid.shape == (nt, nr)
    qadj = np.zeros((nt, ns))
    grad = np.zeros(g.shape) if hist is not None else None
    rc = _L().or_adjoint(ctypes.byref(g._c), _dp(v), _dp(lam), _dp(lamo), nr, _dp(rec.copy()),
                         _dp(resid), ns, _dp(src.copy()), _dp(qadj), nt,
                         _dp(None if hist is None else np.ascontiguousarray(hist)), _dp(grad))
    if rc != 0:
        raise ValueError("sparse point outside the grid")
    return lam, lamo, qadj, grad


def heat(g: Grid, u: np.ndarray, nsteps: int) -> None:
    """Forward-Euler diffusion u <- u + dt Lap u, in place on a padded array."""
    _L().or_heat(ctypes.byref(g._c), _dp(u), nsteps)
