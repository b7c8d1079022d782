"""Pins of the network oracle: library cross-correlation, finite differences,
closed-form GELU values, the first Adam step, BF16 rounding."""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import nn as N


def test_conv3d_is_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 6, 7))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    y = N.conv3d(x, w, b)
    for co in range(4):
        ref = sum(signal.correlate(x[ci], w[co, ci], mode="same") for ci in range(3)) + b[co]
        np.testing.assert_allclose(y[co], ref, rtol=1e-12, atol=1e-12)


def test_conv3d_dgrad_wgrad_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    gy = rng.standard_normal((3, 4, 3, 5))
    f = lambda xx, ww, bb: np.sum(gy * N.conv3d(xx, ww, bb))
    gx = N.conv3d_dgrad(gy, w)
    gw, gb = N.conv3d_wgrad(x, gy)
    eps = 1e-6
    for idx in [(0, 1, 2, 3), (1, 0, 0, 0), (1, 3, 2, 4)]:
        d = np.zeros_like(x)
        d[idx] = eps
        fd = (f(x + d, w, b) - f(x - d, w, b)) / (2 * eps)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1, abs(fd))
    for idx in [(0, 1, 0, 2, 1), (2, 0, 1, 1, 1), (1, 1, 2, 0, 2)]:
        d = np.zeros_like(w)
        d[idx] = eps
        fd = (f(x, w + d, b) - f(x, w - d, b)) / (2 * eps)
        assert abs(fd - gw[idx]) <= 1e-6 * max(1, abs(fd))
    np.testing.assert_allclose(gb, gy.sum(axis=(1, 2, 3)))


def test_gelu_values_and_derivative():
    # GELU(0) = 0, GELU(x) -> x for large x, GELU(-x) = GELU(x) - x
    assert N.gelu(np.array(0.0)) == 0.0
    assert abs(N.gelu(np.array(8.0)) - 8.0) < 1e-12
    x = np.linspace(-4, 4, 33)
    np.testing.assert_allclose(N.gelu(-x), N.gelu(x) - x, atol=1e-14)
    # Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(N.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    h = 1e-6
    np.testing.assert_allclose(N.gelu_grad(x), (N.gelu(x + h) - N.gelu(x - h)) / (2 * h),
                               rtol=1e-7, atol=1e-9)


def test_network_gradients_finite_differences():
    rng = np.random.default_rng(2)
    shapes = [(16, 3, 3, 3, 3), (16,), (16, 16, 3, 3, 3), (16,), (1, 16, 3, 3, 3), (1,)]
    p = [rng.standard_normal(s) * 0.2 for s in shapes]
    net = N.Net(*p)
    x = rng.standard_normal((3, 4, 4, 3))
    t = rng.standard_normal((1, 4, 4, 3))
    loss, grads = net.loss_and_grads(x, t)
    eps = 1e-6
    for k, idx in [(0, (3, 1, 0, 2, 1)), (1, (5,)), (2, (7, 9, 1, 1, 0)), (3, (15,)),
                   (4, (0, 4, 2, 2, 2)), (5, (0,))]:
        pp = [a.copy() for a in p]
        pm = [a.copy() for a in p]
        pp[k][idx] += eps
        pm[k][idx] -= eps
        fd = (N.Net(*pp).loss_and_grads(x, t)[0] - N.Net(*pm).loss_and_grads(x, t)[0]) / (2 * eps)
        assert abs(fd - grads[k][idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, fd, grads[k][idx])


def test_adam_first_step_is_signed_lr():
    """With m0 = v0 = 0, the bias-corrected first update is -lr * g/(|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = N.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-8)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_two_steps_worked_by_hand():
    """Kingma & Ba, Algorithm 1, worked by hand for p0 = 1, gradients 2 then
    -1, lr 0.1, beta1 0.9, beta2 0.999, eps 0:
      t=1: m = 0.2, v = 0.004, m^ = 2, v^ = 4, p = 1 - 0.1 * 2/2 = 0.9;
      t=2: m = 0.18 - 0.1 = 0.08, v = 0.003996 + 0.001 = 0.004996,
           m^ = 0.08/0.19 = 8/19, v^ = 0.004996/0.001999 = 4996/1999,
           p = 0.9 - 0.1 * (8/19) / sqrt(4996/1999).
    Swapping the betas, using the other moment's bias correction, or
    correcting with the step index off by one each changes p2."""
    p, m, v = N.adam_step(np.array([1.0]), np.array([2.0]), np.zeros(1), np.zeros(1), 1,
                          lr=0.1, b1=0.9, b2=0.999, eps=0.0)
    assert abs(p[0] - 0.9) < 1e-15 and abs(m[0] - 0.2) < 1e-15 and abs(v[0] - 0.004) < 1e-15
    p, m, v = N.adam_step(p, np.array([-1.0]), m, v, 2, lr=0.1, b1=0.9, b2=0.999, eps=0.0)
    assert abs(m[0] - 0.08) < 1e-15 and abs(v[0] - 0.004996) < 1e-15
    want = 0.9 - 0.1 * (8.0 / 19.0) / math.sqrt(4996.0 / 1999.0)
    assert abs(p[0] - want) < 1e-14, (p[0], want)
    assert abs(want - 0.873366) < 1e-6


def test_bf16_rounding():
    a = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.1415926, 65504.0, 1e-40],
                 dtype=np.float32)
    r = N.bf16_round(a)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1.0 + 2 ** -7            # above the tie -> up
    assert abs(r[3] + 3.140625) < 1e-12
    assert r[4] == 65536.0
    # representable bf16 values are fixed points
    np.testing.assert_array_equal(N.bf16_round(r.astype(np.float32)), r)


def test_masked_mse_is_subset_sum_over_all_points():
    """Masked points drop out of the sum but stay in the denominator; an empty
    box is the plain MSE, a box over everything gives zero."""
    rng = np.random.default_rng(5)
    y, t = rng.standard_normal((2, 5, 6, 7))
    m = N.box_mask(y.shape, (1, 2, 3), (3, 5, 6))
    keep = np.ones(y.shape, bool)
    keep[1:3, 2:5, 3:6] = False
    assert keep.sum() == y.size - 2 * 3 * 3
    ref = sum(float(d) ** 2 for d in (y - t)[keep]) / y.size
    assert abs(N.masked_mse(y, t, m) - ref) <= 1e-14 * ref
    assert N.masked_mse(y, t, N.box_mask(y.shape)) == N.mse(y, t)
    assert N.masked_mse(y, t, N.box_mask(y.shape, (0, 0, 0), y.shape)) == 0.0


def test_masked_network_gradients_finite_differences():
    """Gradients of the masked loss match central differences, and a parameter
    that only reaches masked outputs gets none of their error."""
    rng = np.random.default_rng(6)
    shapes = [(16, 3, 3, 3, 3), (16,), (16, 16, 3, 3, 3), (16,), (1, 16, 3, 3, 3), (1,)]
    p = [rng.standard_normal(s) * 0.2 for s in shapes]
    x = rng.standard_normal((3, 5, 4, 4))
    t = rng.standard_normal((1, 5, 4, 4))
    mask = N.box_mask((5, 4, 4), (1, 0, 1), (4, 3, 3))[None]
    loss, grads = N.Net(*p).loss_and_grads(x, t, mask)
    eps = 1e-6
    for k, idx in [(0, (2, 2, 1, 0, 2)), (2, (4, 11, 2, 1, 1)), (4, (0, 9, 0, 2, 1)), (5, (0,))]:
        pp = [a.copy() for a in p]
        pm = [a.copy() for a in p]
        pp[k][idx] += eps
        pm[k][idx] -= eps
        fd = (N.Net(*pp).loss_and_grads(x, t, mask)[0] -
              N.Net(*pm).loss_and_grads(x, t, mask)[0]) / (2 * eps)
        assert abs(fd - grads[k][idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, fd, grads[k][idx])
    # the output bias gradient is 2 * sum over unmasked points of (y - t) / N
    y = N.Net(*p).forward(x)
    ref = 2.0 * float(np.sum(mask * (y - t))) / y.size
    assert abs(grads[5][0] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_input_channels_modulated_channel_vanishes_with_field():
    rng = np.random.default_rng(7)
    a, b, c = rng.standard_normal((3, 4, 3, 5))
    a[1] = 0.0
    x = N.input_channels(a, b, c, 2.0, c_times_a=True)
    assert np.all(x[2][1] == 0.0)
    # homogeneous of degree zero in (a, b, s)
    np.testing.assert_allclose(N.input_channels(3 * a, 3 * b, c, 6.0, True), x, rtol=1e-15)
    np.testing.assert_array_equal(N.input_channels(a, b, c, 2.0)[2], c)


def test_adam_frozen_entries_are_untouched():
    g = np.array([0.3, -2.0, 1e-3, 4.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    m0 = np.array([0.1, 0.0, -0.2, 0.0])
    v0 = np.array([0.01, 0.0, 0.04, 0.0])
    fz = np.array([False, True, False, True])
    p, m, v = N.adam_step(p0, g, m0, v0, 3, lr=0.01, frozen=fz)
    pf, mf, vf = N.adam_step(p0, g, m0, v0, 3, lr=0.01)
    np.testing.assert_array_equal(p[fz], p0[fz])
    np.testing.assert_array_equal(m[fz], m0[fz])
    np.testing.assert_array_equal(v[fz], v0[fz])
    np.testing.assert_array_equal(p[~fz], pf[~fz])
    np.testing.assert_array_equal(m[~fz], mf[~fz])
