"""FP64 oracle of the learned-correction network (test infrastructure only).

The network is not in the paper: it is the learned coarse-grid correction
this project adds around the propagator.  Every function here is the plain
textbook definition, evaluated in float64 with numpy:

* conv3d: cross-correlation with a 3x3x3 kernel and zero "same" padding,
      out[co, z, y, x] = b[co] + sum_{ci, dz, dy, dx} w[co, ci, dz, dy, dx]
                                   * in[ci, z+dz-1, y+dy-1, x+dx-1]
  (channels-first arrays [C][nz][ny][nx]);
* its data gradient (the adjoint correlation) and weight/bias gradients;
* GELU(x) = x Phi(x) with the Gaussian CDF Phi (erf form) and its derivative;
* mean-squared error, optionally with points of an index box excluded;
* the input channels (two fields scaled by 1/s and a third channel that is
  either given or modulates the first field);
* one Adam step (Kingma & Ba) with bias correction, optionally leaving some
  entries (the biases of a bias-free network) untouched.

Operands of the BF16 kernels are first rounded to BF16 (round to nearest
even) with ``bf16_round`` and then computed here in float64, so a comparison
measures only the kernels' FP32 accumulation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float64)


def _taps():
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                yield dz, dy, dx


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """x [ci][nz][ny][nx], w [co][ci][3][3][3], b [co] -> [co][nz][ny][nx]."""
    ci, nz, ny, nx = x.shape
    co = w.shape[0]
    xp = np.zeros((ci, nz + 2, ny + 2, nx + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((co, nz, ny, nx))
    for dz, dy, dx in _taps():
        patch = xp[:, dz:dz + nz, dy:dy + ny, dx:dx + nx]          # [ci][...]
        out += np.tensordot(w[:, :, dz, dy, dx], patch, axes=([1], [0]))
    if b is not None:
        out += b[:, None, None, None]
    return out


def conv3d_dgrad(gy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d(sum gy * conv3d(x, w))/dx: gy [co][...], w [co][ci][3][3][3] -> [ci][...]."""
    co, nz, ny, nx = gy.shape
    ci = w.shape[1]
    gx = np.zeros((ci, nz + 2, ny + 2, nx + 2))
    for dz, dy, dx in _taps():
        gx[:, dz:dz + nz, dy:dy + ny, dx:dx + nx] += np.tensordot(
            w[:, :, dz, dy, dx], gy, axes=([0], [0]))
    return gx[:, 1:-1, 1:-1, 1:-1]


def conv3d_wgrad(x: np.ndarray, gy: np.ndarray):
    """(dW, db) of sum gy * conv3d(x, w, b)."""
    ci, nz, ny, nx = x.shape
    co = gy.shape[0]
    xp = np.zeros((ci, nz + 2, ny + 2, nx + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gw = np.zeros((co, ci, 3, 3, 3))
    for dz, dy, dx in _taps():
        patch = xp[:, dz:dz + nz, dy:dy + ny, dx:dx + nx]
        gw[:, :, dz, dy, dx] = np.tensordot(gy, patch, axes=([1, 2, 3], [1, 2, 3]))
    gb = gy.sum(axis=(1, 2, 3))
    return gw, gb


def gelu(x: np.ndarray) -> np.ndarray:
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x: np.ndarray) -> np.ndarray:
    """d GELU / dx = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def mse(pred: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((pred - target) ** 2))


def box_mask(shape, lo=None, hi=None) -> np.ndarray:
    """1 everywhere except 0 inside the half-open index box [lo, hi)."""
    m = np.ones(shape)
    if lo is not None:
        m[tuple(slice(int(a), int(b)) for a, b in zip(lo, hi))] = 0.0
    return m


def masked_mse(pred: np.ndarray, target: np.ndarray, mask: np.ndarray) -> float:
    """Sum of mask * squared error divided by the number of ALL points (the
    masked points count in the denominator and contribute zero)."""
    return float(np.sum(mask * (pred - target) ** 2) / pred.size)


def input_channels(a, b, c, s=1.0, c_times_a=False) -> np.ndarray:
    """Network input [3][...]: (a/s, b/s, c*a/s) or (a/s, b/s, c)."""
    a = np.asarray(a, dtype=np.float64) / s
    b = np.asarray(b, dtype=np.float64) / s
    c = np.asarray(c, dtype=np.float64)
    return np.stack([a, b, c * a if c_times_a else c])


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, frozen=None):
    """One Adam update at step t (1-based).  Returns (p, m, v).  Entries
    where the boolean array `frozen` is true keep p, m and v unchanged."""
    m1 = b1 * m + (1 - b1) * g
    v1 = b2 * v + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** t)
    vh = v1 / (1 - b2 ** t)
    p1 = p - lr * mh / (np.sqrt(vh) + eps)
    if frozen is not None:
        p1, m1, v1 = (np.where(frozen, a0, a1) for a0, a1 in ((p, p1), (m, m1), (v, v1)))
    return p1, m1, v1


def _keep(a):
    return a


class Net:
    """conv(3->16) - GELU - conv(16->16) - GELU - conv(16->1), 3^3 kernels.

    ``store`` (default: none) is a rounding applied wherever a stored
    activation or gradient is formed: the pre-activations z1, z2, the
    activations GELU(z1), GELU(z2) (each evaluated on the rounded
    pre-activation), the output gradient dL/dy and the back-propagated
    gradients dL/dz2, dL/dz1.  With ``store=bf16_round`` the network keeps
    exactly the BF16 tensors a BF16-storage implementation keeps; y, the loss
    and the parameter gradients stay in float64.  Without it this is the
    plain textbook network (pinned by finite differences)."""

    def __init__(self, w1, b1, w2, b2, w3, b3, store=None):
        self.p = [np.asarray(a, dtype=np.float64) for a in (w1, b1, w2, b2, w3, b3)]
        self.store = store or _keep

    def forward(self, x, keep=False):
        w1, b1, w2, b2, w3, b3 = self.p
        st = self.store
        z1 = st(conv3d(x, w1, b1))
        a1 = st(gelu(z1))
        z2 = st(conv3d(a1, w2, b2))
        a2 = st(gelu(z2))
        y = conv3d(a2, w3, b3)
        if keep:
            return y, (x, z1, a1, z2, a2)
        return y

    def loss_and_grads(self, x, target, mask=None):
        """MSE over all outputs (masked_mse when a 0/1 mask of the output's
        shape is given) and its gradient w.r.t. every parameter."""
        w1, b1, w2, b2, w3, b3 = self.p
        y, (x, z1, a1, z2, a2) = self.forward(x, keep=True)
        n = y.size
        m = np.ones_like(y) if mask is None else np.broadcast_to(mask, y.shape)
        st = self.store
        gy = st(2.0 * m * (y - target) / n)
        gw3, gb3 = conv3d_wgrad(a2, gy)
        ga2 = conv3d_dgrad(gy, w3)
        gz2 = st(ga2 * gelu_grad(z2))
        gw2, gb2 = conv3d_wgrad(a1, gz2)
        ga1 = conv3d_dgrad(gz2, w2)
        gz1 = st(ga1 * gelu_grad(z1))
        gw1, gb1 = conv3d_wgrad(x, gz1)
        return masked_mse(y, target, m), [gw1, gb1, gw2, gb2, gw3, gb3]
