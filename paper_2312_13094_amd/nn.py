"""ctypes binding to the learned-correction network kernels (include/fdnn.h).

Argument marshalling only: convolutions, GELU, loss, gradients and Adam all
run in libfd.so.  ``Net`` owns the caller-side device buffers (FP32 master
parameters, Adam moments, packed BF16 fragments, activations) as torch
tensors and sequences the library calls for inference and training.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import fd as FD


class View(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("pitch_y", ctypes.c_int64),
                ("pitch_z", ctypes.c_int64)]


class Box(ctypes.Structure):
    """Half-open (z, y, x) index box [lo, hi)."""
    _fields_ = [("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3)]


def box(lo, hi):
    return Box((ctypes.c_int * 3)(*[int(v) for v in lo]), (ctypes.c_int * 3)(*[int(v) for v in hi]))


def _bp(b):
    return None if b is None else ctypes.byref(b)


def dense_view(shape):
    nz, ny, nx = shape
    return View(0, nx, ny * nx)


def grid_view(grid):
    L = grid.layout
    return View(int(L.offset), int(L.pitch_y), int(L.pitch_z))


_bound = False


def lib():
    global _bound
    L = FD.lib()
    if not _bound:
        vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.nn_param_count.restype = ctypes.c_int64
        L.nn_packed_bytes.restype = ctypes.c_int64
        L.nn_rms_scratch_floats.restype = ctypes.c_int64
        L.nn_wgrad_workspace_bytes.restype = ctypes.c_int64
        L.nn_wgrad_workspace_bytes.argtypes = [i, i, i]
        L.nn_pack_weights.argtypes = [vp, vp, vp]
        L.nn_pack_input.argtypes = [i, i, i, vp, View, vp, View, vp, View, i, vp, vp, vp]
        L.nn_rms.argtypes = [i, i, i, vp, View, vp, vp, vp]
        L.nn_conv_gelu.argtypes = [i, i, i, i, vp, vp, vp, vp, vp, vp]
        L.nn_conv_gelu_fields.argtypes = [i, i, i, vp, View, vp, View, vp, View, i, vp, vp, vp,
                                          vp, vp, vp]
        bp = ctypes.POINTER(Box)
        L.nn_conv_out.argtypes = [i, i, i, vp, vp, vp, vp, vp, View, vp, View, vp, f, bp, vp]
        L.nn_mse.argtypes = [i, i, i, vp, vp, vp, f, bp, vp, vp, vp]
        L.nn_dgrad_gelu.argtypes = [i, i, i, i, vp, vp, vp, vp, vp]
        L.nn_wgrad.argtypes = [i, i, i, i, vp, vp, vp, vp, i, vp]
        L.nn_wgrad_noalloc.argtypes = [i, i, i, i, vp, vp, vp, i, vp]
        L.nn_adam.argtypes = [vp, vp, vp, vp, i, f, f, f, f, i, vp]
        _bound = True
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _chk(rc):
    FD._check(rc)


PARAM_SHAPES = [(16, 3, 27), (16,), (16, 16, 27), (16,), (1, 16, 27), (1,)]


def init_params(seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """He-style random init (FP32, the library's flat layout); the output layer
    starts small so the untrained correction is close to zero."""
    rng = np.random.default_rng(seed)
    out = []
    for k, s in enumerate(PARAM_SHAPES):
        if len(s) == 1:
            out.append(np.zeros(s))
        else:
            fan_in = s[1] * 27
            std = gain * np.sqrt(2.0 / fan_in) * (0.05 if k == 4 else 1.0)
            out.append(rng.standard_normal(s) * std)
    flat = np.concatenate([a.ravel() for a in out]).astype(np.float32)
    assert flat.size == lib().nn_param_count()
    return flat


def split_params(flat):
    """Flat parameter vector -> [w1, b1, w2, b2, w3, b3] in the oracle's shapes."""
    out, o = [], 0
    for s in PARAM_SHAPES:
        n = int(np.prod(s))
        a = flat[o:o + n]
        if len(s) == 3:
            a = a.reshape(s[0], s[1], 3, 3, 3)
        out.append(a)
        o += n
    return out


class Net:
    """Device state of the 3-layer correction network for volumes of `shape`."""

    def __init__(self, shape, params=None, device=0, bias=True):
        """bias=False: biases stay at their initial values (zero from
        init_params) during training."""
        self.shape = tuple(int(v) for v in shape)
        self.train_bias = bool(bias)
        self.dev = torch.device("cuda", device)
        L = lib()
        n = int(np.prod(self.shape))
        P = params if params is not None else init_params()
        self.params = torch.from_numpy(np.asarray(P, dtype=np.float32)).to(self.dev)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.packed = torch.zeros(int(L.nn_packed_bytes()) // 2, dtype=torch.int16, device=self.dev)
        u16 = dict(dtype=torch.int16, device=self.dev)
        self.x8 = torch.zeros(n * 8, **u16)
        self.z1 = torch.zeros(n * 16, **u16)
        self.a1 = torch.zeros(n * 16, **u16)
        self.z2 = torch.zeros(n * 16, **u16)
        self.a2 = torch.zeros(n * 16, **u16)
        self.g8 = torch.zeros(n * 8, **u16)
        self.g16a = torch.zeros(n * 16, **u16)
        self.g16b = torch.zeros(n * 16, **u16)
        self.y = torch.zeros(n, dtype=torch.float32, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        self.scale = torch.zeros(int(L.nn_rms_scratch_floats()), dtype=torch.float32,
                                 device=self.dev)
        self.flag = torch.zeros(1, dtype=torch.int32, device=self.dev)
        ws = int(L.nn_wgrad_workspace_bytes(*self.shape))
        self.ws = torch.zeros(ws // 4, dtype=torch.float32, device=self.dev)
        self.pack()

    # -- parameters ----------------------------------------------------------
    def pack(self):
        _chk(lib().nn_pack_weights(_p(self.params), _p(self.packed), _s()))

    def set_params(self, flat):
        self.params.copy_(torch.as_tensor(np.asarray(flat, dtype=np.float32)))
        self.pack()

    # -- building blocks -----------------------------------------------------
    def pack_input(self, a, va, b, vb, c, vc, scale=None, c_times_a=False):
        nz, ny, nx = self.shape
        _chk(lib().nn_pack_input(nz, ny, nx, _p(a), va, _p(b), vb, _p(c), vc, int(c_times_a),
                                 _p(scale), _p(self.x8), _s()))

    def rms(self, u, vu, scale=None):
        """RMS of u into scale[0] (scale: nn_rms_scratch_floats() floats;
        self.scale if None)."""
        nz, ny, nx = self.shape
        _chk(lib().nn_rms(nz, ny, nx, _p(u), vu, _p(self.scale if scale is None else scale),
                          _p(self.flag), _s()))

    def forward(self, keep=True, out=None, base=None, vbase=None, vout=None, scale=None,
                ydense=True, gain=1.0, skip=None, fields=None):
        """Layers 1-3 on self.x8, or, with fields = (a, va, b, vb, c, vc,
        c_times_a), on the input pack_input(a, va, b, vb, c, vc, scale,
        c_times_a) would write, formed inside layer 1 (bitwise the same).
        keep: store pre-activations (training)."""
        nz, ny, nx = self.shape
        L = lib()
        if fields is None:
            _chk(L.nn_conv_gelu(1, nz, ny, nx, _p(self.x8), _p(self.packed), _p(self.params),
                                _p(self.z1) if keep else None, _p(self.a1), _s()))
        else:
            a, va, b, vb, c, vc, cta = fields
            _chk(L.nn_conv_gelu_fields(nz, ny, nx, _p(a), va, _p(b), vb, _p(c), vc, int(cta),
                                       _p(scale), _p(self.packed), _p(self.params),
                                       _p(self.z1) if keep else None, _p(self.a1), _s()))
        _chk(L.nn_conv_gelu(2, nz, ny, nx, _p(self.a1), _p(self.packed), _p(self.params),
                            _p(self.z2) if keep else None, _p(self.a2), _s()))
        dv = dense_view(self.shape)
        _chk(L.nn_conv_out(nz, ny, nx, _p(self.a2), _p(self.packed), _p(self.params),
                           _p(self.y) if ydense else None, _p(base), vbase or dv, _p(out),
                           vout or dv, _p(scale), float(gain), _bp(skip), _s()))

    def backward(self, target, scale=None, gain=1.0, skip=None, accumulate=False):
        """MSE against target / (gain * scale[0]) (dense FP32, zero weight
        inside `skip`) and all parameter gradients (added to self.grads if
        accumulate)."""
        acc = int(accumulate)
        nz, ny, nx = self.shape
        L = lib()
        _chk(L.nn_mse(nz, ny, nx, _p(self.y), _p(target), _p(scale), float(gain), _bp(skip),
                      _p(self.g8), _p(self.loss), _s()))
        _chk(L.nn_wgrad(3, nz, ny, nx, _p(self.a2), _p(self.g8), _p(self.ws), _p(self.grads), acc,
                        _s()))
        _chk(L.nn_dgrad_gelu(3, nz, ny, nx, _p(self.g8), _p(self.packed), _p(self.z2),
                             _p(self.g16a), _s()))
        _chk(L.nn_wgrad(2, nz, ny, nx, _p(self.a1), _p(self.g16a), _p(self.ws), _p(self.grads),
                        acc, _s()))
        _chk(L.nn_dgrad_gelu(2, nz, ny, nx, _p(self.g16a), _p(self.packed), _p(self.z1),
                             _p(self.g16b), _s()))
        _chk(L.nn_wgrad(1, nz, ny, nx, _p(self.x8), _p(self.g16b), _p(self.ws), _p(self.grads),
                        acc, _s()))

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _chk(lib().nn_adam(_p(self.params), _p(self.grads), _p(self.m), _p(self.v), self.t,
                           lr, b1, b2, eps, int(self.train_bias), _s()))
        self.pack()
