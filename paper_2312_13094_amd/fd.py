"""Thin ctypes binding to libfd (``include/fd.h``).

Argument marshalling only: every step of the propagation runs in the HIP
kernels of ``libfd.so``.  PyTorch provides device memory (tensors whose
``data_ptr()`` is passed through) and the stream (the current torch stream).
There is no fallback: if the library is missing, importing this module's
loader raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfd.so")

FD_OK, FD_EINVAL, FD_ENOMEM, FD_EDEVICE, FD_EUNSTABLE, FD_ENOTSUP = 0, -1, -2, -3, -4, -5
FD_ACOUSTIC, FD_TTI, FD_ELASTIC, FD_VISCO = 0, 1, 2, 3
ELASTIC_FIELDS = ("vx", "vy", "vz", "txx", "tyy", "tzz", "txy", "txz", "tyz")
VISCO_FIELDS = ELASTIC_FIELDS + ("rxx", "ryy", "rzz", "rxy", "rxz", "ryz")
FD_BC_ZERO, FD_BC_LOOPBACK, FD_BC_EXTERNAL = 0, 1, 2
FD_XCHG_BASIC, FD_XCHG_FULL = 0, 1
ALL_FACES = 0x3F


class FdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libfd error %d: %s" % (code, msg))
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("shape", ctypes.c_int64 * 3),
                ("spacing", ctypes.c_double * 3), ("space_order", ctypes.c_int),
                ("nbl", ctypes.c_int), ("physics", ctypes.c_int), ("boundary", ctypes.c_int),
                ("dt", ctypes.c_double), ("vmax", ctypes.c_double), ("eps_max", ctypes.c_double),
                ("device", ctypes.c_int)]


class Layout(ctypes.Structure):
    _fields_ = [("padded", ctypes.c_int64 * 3), ("pitch_y", ctypes.c_int64),
                ("pitch_z", ctypes.c_int64), ("offset", ctypes.c_int64), ("halo", ctypes.c_int),
                ("field_elems", ctypes.c_int64), ("field_bytes", ctypes.c_size_t)]


class SparseC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("base_dev", ctypes.c_void_p), ("frac_dev", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libfd.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfd.so is not built (python -m paper_2312_13094_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    P = ctypes.POINTER
    L.fd_create_grid.argtypes = [P(GridDesc), P(vp)]
    L.fd_destroy_grid.argtypes = [vp]
    L.fd_destroy_grid.restype = None
    L.fd_field_layout.argtypes = [vp, P(Layout)]
    L.fd_set_tile.argtypes = [vp, i, i, i, i]
    L.fd_set_exchange_mode.argtypes = [vp, i]
    L.fd_sparse_prepare.argtypes = [vp, P(ctypes.c_double), i, P(ctypes.c_int32),
                                    P(ctypes.c_float)]
    L.fd_set_model.argtypes = [vp, vp, P(vp), vp]
    L.fd_forward.argtypes = [vp, P(vp), P(SparseC), vp, P(SparseC), vp, i, P(vp), i, vp]
    L.fd_adjoint.argtypes = [vp, P(vp), P(SparseC), vp, P(SparseC), vp, vp, i, P(vp), i, P(vp),
                             vp, vp]
    L.fd_step.argtypes = [vp, vp, vp, P(SparseC), vp, P(SparseC), vp, vp]
    L.fd_step_lagged.argtypes = [vp, vp, vp, P(SparseC), vp, P(SparseC), vp, vp]
    L.fd_gradient_to_velocity.argtypes = [vp, vp, vp, vp]
    L.fd_sample.argtypes = [vp, vp, P(SparseC), vp, vp]
    L.fd_autotune.argtypes = [vp, ctypes.c_char_p, P(ctypes.c_int), P(ctypes.c_double), vp]
    L.fd_halo_face_elems.argtypes = [vp, i]
    L.fd_halo_face_elems.restype = i64
    L.fd_pack_halo.argtypes = [vp, vp, ctypes.c_uint, P(vp), vp]
    L.fd_unpack_halo.argtypes = [vp, vp, ctypes.c_uint, P(vp), vp]
    L.fd_copy_floats.argtypes = [vp, vp, i64, vp]
    L.fd_profile_begin.argtypes = [vp, i]
    L.fd_profile_end.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int)]
    L.fd_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != FD_OK:
        raise FdError(rc, lib().fd_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts, need=0, what="pointer array"):
    """A C array of device pointers.  The library reads a fixed number of
    entries from it (given by the call and the handle), so a shorter list
    is rejected here: reading past its end would pass stray addresses to
    the kernels."""
    if ts is None:
        return None
    if len(ts) < need:
        raise FdError(FD_EINVAL, "%s: %d device arrays needed, %d given" % (what, need, len(ts)))
    arr = (ctypes.c_void_p * len(ts))()
    for k, t in enumerate(ts):
        arr[k] = None if t is None else t.data_ptr()
    return arr


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def copy_floats(dst, src, n=None):
    """Device copy of n floats with the library's copy kernel."""
    n = dst.numel() if n is None else n
    _check(lib().fd_copy_floats(_ptr(dst), _ptr(src), int(n), _stream(dst.device.index or 0)))


class SparsePoints:
    """Prepared sparse points resident on the device."""

    def __init__(self, grid, coords):
        import torch
        coords = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, grid.ndim)
        n = coords.shape[0]
        base = np.zeros((max(n, 1), grid.ndim), dtype=np.int32)
        frac = np.zeros((max(n, 1), grid.ndim), dtype=np.float32)
        _check(lib().fd_sparse_prepare(
            grid.handle, coords.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
            base.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            frac.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        self.n = n
        self.base_host, self.frac_host = base[:n], frac[:n]
        dev = grid.torch_device
        self.base = torch.from_numpy(base).to(dev)
        self.frac = torch.from_numpy(frac).to(dev)
        self.c = SparseC(n, self.base.data_ptr(), self.frac.data_ptr())


class Grid:
    """One subdomain handle (``fd_grid``)."""

    def __init__(self, shape, spacing, so, dt, vmax, nbl=0, boundary=FD_BC_ZERO,
                 physics=FD_ACOUSTIC, eps_max=0.0, device=0):
        self.ndim = len(shape)
        self.shape = tuple(int(s) for s in shape)
        self.spacing = tuple(float(h) for h in spacing)
        self.so, self.dt, self.vmax, self.nbl = so, dt, vmax, nbl
        self.boundary, self.physics, self.device = boundary, physics, device
        d = GridDesc()
        d.ndim = self.ndim
        for k in range(self.ndim):
            d.shape[k] = self.shape[k]
            d.spacing[k] = self.spacing[k]
        d.space_order, d.nbl, d.physics, d.boundary = so, nbl, physics, boundary
        d.dt, d.vmax, d.eps_max, d.device = dt, vmax, eps_max, device
        self.desc = d
        h = ctypes.c_void_p()
        _check(lib().fd_create_grid(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        L = Layout()
        _check(lib().fd_field_layout(h, ctypes.byref(L)))
        self.layout = L

    # -- memory helpers ------------------------------------------------------
    @property
    def torch_device(self):
        import torch
        return torch.device("cuda", self.device)

    @property
    def field_elems(self):
        return int(self.layout.field_elems)

    def field(self):
        """A zeroed padded field (1-D float32 device tensor)."""
        import torch
        return torch.zeros(self.field_elems, dtype=torch.float32, device=self.torch_device)

    def _dims(self):
        L = self.layout
        if self.ndim == 3:
            return self.shape, (int(L.pitch_z), int(L.pitch_y), 1)
        return self.shape, (int(L.pitch_z), 1)

    def domain(self, f):
        """DOMAIN view (z, [y,] x) of a padded field."""
        shp, st = self._dims()
        return f.as_strided(shp, st, int(self.layout.offset))

    def with_halo(self, f):
        """DOMAIN + halo view of a padded field."""
        r = int(self.layout.halo)
        shp, st = self._dims()
        shp = tuple(s + 2 * r for s in shp)
        off = int(self.layout.offset) - r * sum(st)
        return f.as_strided(shp, st, off)

    def face_elems(self, f):
        return int(lib().fd_halo_face_elems(self.handle, f))

    # -- API -----------------------------------------------------------------
    def set_tile(self, by, ry=1, nzb=64, xcd=1):
        _check(lib().fd_set_tile(self.handle, by, ry, nzb, xcd))

    def set_exchange_mode(self, mode):
        """FD_XCHG_BASIC (exchange, then step) or FD_XCHG_FULL (exchange on a
        second stream overlapped with the CORE, then the REMAINDER)."""
        _check(lib().fd_set_exchange_mode(self.handle, mode))

    def autotune(self, cache_path=None):
        """Timed tile search (or cache lookup); returns ((by, ry, nzb, xcd), ms)."""
        t = (ctypes.c_int * 4)()
        ms = ctypes.c_double()
        _check(lib().fd_autotune(self.handle, cache_path.encode() if cache_path else None, t,
                                 ctypes.byref(ms), _stream(self.device)))
        return tuple(t), ms.value

    def sparse(self, coords):
        return SparsePoints(self, coords)

    # device arrays a call reads per physics: model aux fields, state fields
    _AUX = {FD_ACOUSTIC: 0, FD_TTI: 4, FD_ELASTIC: 2, FD_VISCO: 5}
    _NSTATE = {FD_ACOUSTIC: 2, FD_TTI: 4, FD_ELASTIC: 9, FD_VISCO: 15}

    def set_model(self, vel, tti=None):
        """vel plus the physics' aux fields: TTI {eps, delta, theta, phi},
        elastic {vs, rho}, visco-elastic {vs, rho, tau_ep, tau_es, tau_s}."""
        need = self._AUX[self.physics]
        if tti is not None and len(tti) != need:
            raise FdError(FD_EINVAL, "set_model: %d aux fields for this physics, %d given"
                          % (need, len(tti)))
        arr = _ptr_array(tti, need, "set_model") if tti is not None else None
        _check(lib().fd_set_model(self.handle, _ptr(vel), arr, _stream(self.device)))

    def _ckpt_need(self, nstate, nt, ckpt, every):
        if ckpt is None or every < 1:
            return 0
        return nstate * ((int(nt) + every - 1) // every)

    def forward(self, states, src=None, q=None, rec=None, d=None, nt=0, ckpt=None,
                ckpt_every=0):
        ns = self._NSTATE[self.physics]
        _check(lib().fd_forward(
            self.handle, _ptr_array(states, ns, "forward states"),
            ctypes.byref(src.c) if src else None, _ptr(q),
            ctypes.byref(rec.c) if rec else None, _ptr(d), int(nt),
            _ptr_array(ckpt, self._ckpt_need(ns, nt, ckpt, int(ckpt_every)), "checkpoints"),
            int(ckpt_every), _stream(self.device)))

    def adjoint(self, states, rec=None, resid=None, src=None, q=None, qadj=None, nt=0,
                ckpt=None, ckpt_every=0, slots=None, grad_m=None):
        k = int(ckpt_every)
        _check(lib().fd_adjoint(
            self.handle, _ptr_array(states, 2, "adjoint states"),
            ctypes.byref(rec.c) if rec else None, _ptr(resid),
            ctypes.byref(src.c) if src else None, _ptr(q), _ptr(qadj), int(nt),
            _ptr_array(ckpt, self._ckpt_need(2, nt, ckpt, k), "checkpoints"), k,
            _ptr_array(slots, k + 2 if grad_m is not None and k >= 1 else 0, "slots"),
            _ptr(grad_m), _stream(self.device)))

    def step(self, u, um_up, src=None, q=None, rec=None, d=None, lagged=False):
        """One update in place: um_up (u^(n-1)) becomes u^(n+1); q, d are this
        update's source values and receiver outputs (lagged: d records u, the
        level the update reads, instead of the new one)."""
        fn = lib().fd_step_lagged if lagged else lib().fd_step
        _check(fn(
            self.handle, _ptr(u), _ptr(um_up), ctypes.byref(src.c) if src else None, _ptr(q),
            ctypes.byref(rec.c) if rec else None, _ptr(d), _stream(self.device)))

    def sample(self, field, rec, out):
        _check(lib().fd_sample(self.handle, _ptr(field), ctypes.byref(rec.c), _ptr(out),
                               _stream(self.device)))

    def gradient_to_velocity(self, grad_m, grad_v):
        _check(lib().fd_gradient_to_velocity(self.handle, _ptr(grad_m), _ptr(grad_v),
                                             _stream(self.device)))

    def pack_halo(self, field, bufs, mask=ALL_FACES):
        _check(lib().fd_pack_halo(self.handle, _ptr(field), mask, _ptr_array(bufs, 6, "faces"),
                                  _stream(self.device)))

    def unpack_halo(self, field, bufs, mask=ALL_FACES):
        _check(lib().fd_unpack_halo(self.handle, _ptr(field), mask, _ptr_array(bufs, 6, "faces"),
                                    _stream(self.device)))

    def profile_begin(self, max_launches):
        _check(lib().fd_profile_begin(self.handle, int(max_launches)))

    def profile_end(self):
        """(summed step-kernel milliseconds, launches timed) since profile_begin."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        _check(lib().fd_profile_end(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().fd_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Batched multi-shot gradient (``fd_batch``): uneven apertures advanced
    together, the whole schedule replayed as one graph launch."""

    def __init__(self, spacing, so, dt, vmax, nbl, shapes, origins, full_shape, nt, ckpt_every,
                 device=0):
        L = lib()
        _bind_batch(L)
        d = GridDesc()
        d.ndim = 3
        for k in range(3):
            d.spacing[k] = float(spacing[k])
        d.space_order, d.nbl, d.dt, d.vmax, d.device = so, nbl, dt, vmax, device
        self.nshots = len(shapes)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.origins = [tuple(int(v) for v in o) for o in origins]
        self.full_shape = tuple(int(v) for v in full_shape)
        self.nt, self.device = nt, device
        sh = (ctypes.c_int64 * (3 * self.nshots))(*[v for s in self.shapes for v in s])
        og = (ctypes.c_int64 * (3 * self.nshots))(*[v for o in self.origins for v in o])
        fs = (ctypes.c_int64 * 3)(*self.full_shape)
        h = ctypes.c_void_p()
        _check(L.fd_batch_create(ctypes.byref(d), self.nshots, sh, og, fs, int(nt),
                                 int(ckpt_every), ctypes.byref(h)))
        self.handle = h
        self.nrec = [0] * self.nshots

    @property
    def device_bytes(self):
        return int(lib().fd_batch_device_bytes(self.handle))

    def set_tile(self, by, ry, nzb, xcd=1):
        _check(lib().fd_batch_set_tile(self.handle, by, ry, nzb, xcd))

    @property
    def tile(self):
        t = (ctypes.c_int * 4)()
        _check(lib().fd_batch_get_tile(self.handle, t))
        return tuple(t)

    def autotune(self, cache_path=None):
        """Timed search of the batched step's tile (or cache lookup); needs a
        loaded model.  Returns ((by, ry, nzb, flags), ms per launch)."""
        t = (ctypes.c_int * 4)()
        ms = ctypes.c_double()
        _check(lib().fd_batch_autotune(self.handle, cache_path.encode() if cache_path else None,
                                       t, ctypes.byref(ms), _stream(self.device)))
        return tuple(t), ms.value

    def set_geometry(self, shot, src, rec):
        src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
        rec = np.ascontiguousarray(rec, dtype=np.float64).reshape(-1, 3)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().fd_batch_set_geometry(self.handle, shot, src.ctypes.data_as(dp), src.shape[0],
                                           rec.ctypes.data_as(dp), rec.shape[0]))
        self.nrec[shot] = rec.shape[0]

    def set_model(self, vel_full):
        self._vel = vel_full
        _check(lib().fd_batch_set_model(self.handle, _ptr(vel_full), _stream(self.device)))

    def gradient(self, q, dobs, d, grad_v):
        n = self.nshots
        _check(lib().fd_batch_gradient(self.handle, _ptr_array(q, n, "q"),
                                       _ptr_array(dobs, n, "dobs"), _ptr_array(d, n, "d"),
                                       _ptr(grad_v), _stream(self.device)))

    def close(self):
        if getattr(self, "handle", None):
            lib().fd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bind_batch(L):
    if getattr(L, "_batch_bound", False):
        return
    vp, i = ctypes.c_void_p, ctypes.c_int
    P = ctypes.POINTER
    L.fd_batch_create.argtypes = [P(GridDesc), i, P(ctypes.c_int64), P(ctypes.c_int64),
                                  P(ctypes.c_int64), i, i, P(vp)]
    L.fd_batch_destroy.argtypes = [vp]
    L.fd_batch_destroy.restype = None
    L.fd_batch_device_bytes.argtypes = [vp]
    L.fd_batch_device_bytes.restype = ctypes.c_size_t
    L.fd_batch_set_tile.argtypes = [vp, i, i, i, i]
    L.fd_batch_get_tile.argtypes = [vp, P(i)]
    L.fd_batch_autotune.argtypes = [vp, ctypes.c_char_p, P(i), P(ctypes.c_double), vp]
    L.fd_batch_set_geometry.argtypes = [vp, i, P(ctypes.c_double), i, P(ctypes.c_double), i]
    L.fd_batch_set_model.argtypes = [vp, vp, vp]
    L.fd_batch_gradient.argtypes = [vp, P(vp), P(vp), P(vp), vp, vp]
    L._batch_bound = True
