"""GPU BF16-MFMA network kernels against the FP64 network oracle evaluated on
the same BF16-rounded operands.  Outputs stored in BF16 are compared within
BF16 rounding (relative L2 <= 5e-3); FP32 outputs (layer-3 output, weight
gradients) within 1e-4 relative L2 (FP32 accumulation order only)."""
import numpy as np
import pytest

from oracle import nn as N
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

# (11, 13, 37): a few conv tiles (32 x 8 columns, 16-plane z chunks) with
# ragged edges, fewer weight-gradient tiles (32 x 4 x 4) than its 512
# persistent blocks.  (48, 68, 70): three z chunks per column tile, ragged in
# x and y, and 612 weight-gradient tiles, so blocks accumulate several tiles
# and the ordered reduction sums full partials.
SHAPES = [(11, 13, 37), (48, 68, 70)]


@pytest.fixture(params=SHAPES, ids=lambda s: "x".join(map(str, s)))
def shape(request):
    return request.param


def _bits(a):
    """float -> BF16 bit patterns (round to nearest even) as int16."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r.view(np.int16)


def _from_bits(t, c, shape):
    """device int16 BF16 bits [n*c] -> float64 [c][nz][ny][nx]"""
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    a = b.view(np.float32).astype(np.float64).reshape(tuple(shape) + (c,))
    return np.moveaxis(a, -1, 0)


def _cl(a):
    """[c][...] -> channels-last flat"""
    return np.ascontiguousarray(np.moveaxis(np.asarray(a), 0, -1)).ravel()


def _net(params, shape):
    from paper_2312_13094_amd import nn
    return nn.Net(shape, params)


def _params(seed=0, scale=0.3):
    from paper_2312_13094_amd import nn
    rng = np.random.default_rng(seed)
    p = nn.init_params(seed, gain=1.0)
    p[1296:1312] = rng.standard_normal(16) * 0.1
    p[8224:8240] = rng.standard_normal(16) * 0.1
    p[8240:8672] *= 20.0 * scale
    p[8672] = 0.05
    return p


def _oracle_params(p):
    from paper_2312_13094_amd import nn
    w1, b1, w2, b2, w3, b3 = nn.split_params(p)
    return (N.bf16_round(w1), b1.astype(np.float64), N.bf16_round(w2), b2.astype(np.float64),
            N.bf16_round(w3), b3.astype(np.float64))


def _input(shape, seed=1):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape).astype(np.float32) for _ in range(3)]


def test_forward_layers_match_oracle(shape):
    import torch
    from paper_2312_13094_amd import nn
    p = _params()
    net = _net(p, shape)
    a, b, c = _input(shape)
    dv = nn.dense_view(shape)
    ta, tb, tc = (torch.from_numpy(v).cuda() for v in (a, b, c))
    net.pack_input(ta, dv, tb, dv, tc, dv)
    net.forward(keep=True)
    torch.cuda.synchronize()
    w1, b1, w2, b2, w3, b3 = _oracle_params(p)
    x = np.stack([N.bf16_round(v) for v in (a, b, c)])
    np.testing.assert_array_equal(_from_bits(net.x8, 8, shape)[:3], x)
    z1 = N.conv3d(x, w1, b1)
    assert rel_l2(_from_bits(net.z1, 16, shape), z1) <= 5e-3
    # the next layers from the oracle's own BF16-rounded activations
    a1 = N.bf16_round(N.gelu(N.bf16_round(z1)))
    assert rel_l2(_from_bits(net.a1, 16, shape), a1) <= 5e-3
    z2 = N.conv3d(a1, w2, b2)
    assert rel_l2(_from_bits(net.z2, 16, shape), z2) <= 1e-2
    a2 = N.bf16_round(N.gelu(N.bf16_round(z2)))
    y = N.conv3d(a2, w3, b3)[0]
    assert rel_l2(net.y.cpu().numpy().reshape(shape), y) <= 2e-2


def test_output_layer_fp32_and_residual(shape):
    """Layer 3 alone on a known BF16 activation: FP32 output within 1e-4, and
    the fused residual update out = base + s * y through a padded view."""
    import torch
    from paper_2312_13094_amd import nn
    p = _params(3)
    net = _net(p, shape)
    rng = np.random.default_rng(4)
    a2 = rng.standard_normal((16,) + shape).astype(np.float32)
    net.a2.copy_(torch.from_numpy(_bits(_cl(a2))))
    L = nn.lib()
    nz, ny, nx = shape
    # padded destination: rows of nx + 11 floats, 2-point margins
    py = nx + 11
    pz = (ny + 4) * py
    off = 2 * pz + 2 * py + 3
    base = torch.from_numpy(rng.standard_normal((nz + 4) * pz).astype(np.float32)).cuda()
    out = torch.full_like(base, 7.0)
    scale = torch.zeros(int(L.nn_rms_scratch_floats()), device="cuda")
    scale[0] = 2.5
    vb = nn.View(off, py, pz)
    nn._chk(L.nn_conv_out(nz, ny, nx, nn._p(net.a2), nn._p(net.packed), nn._p(net.params),
                          nn._p(net.y), nn._p(base), vb, nn._p(out), vb, nn._p(scale), 1.0, None,
                          nn._s()))
    torch.cuda.synchronize()
    w3, b3 = _oracle_params(p)[4:]
    y = N.conv3d(N.bf16_round(a2), w3, b3)[0]
    got = net.y.cpu().numpy().reshape(shape)
    assert rel_l2(got, y) <= 1e-4
    o = out.cpu().numpy()
    bs = base.cpu().numpy()
    idx = off + np.arange(nz)[:, None, None] * pz + np.arange(ny)[None, :, None] * py + \
        np.arange(nx)[None, None, :]
    np.testing.assert_allclose(o[idx], bs[idx] + 2.5 * got, rtol=1e-6, atol=1e-6)
    mask = np.ones(o.size, bool)
    mask[idx.ravel()] = False
    assert np.all(o[mask] == 7.0)
    # gain and an excluded box, updated in place (out aliases base)
    lo, hi = (2, 3, 10), (7, 9, 30)
    bx = nn.box(lo, hi)
    before = base.clone()
    nn._chk(L.nn_conv_out(nz, ny, nx, nn._p(net.a2), nn._p(net.packed), nn._p(net.params),
                          None, nn._p(base), vb, nn._p(base), vb, nn._p(scale), 1e-3,
                          nn._bp(bx), nn._s()))
    torch.cuda.synchronize()
    m = N.box_mask(shape, lo, hi)
    b0 = before.cpu().numpy()[idx]
    np.testing.assert_allclose(base.cpu().numpy()[idx], b0 + 2.5e-3 * m * got, rtol=1e-6,
                               atol=1e-7)
    np.testing.assert_array_equal(base.cpu().numpy()[idx][m == 0], b0[m == 0])
    np.testing.assert_array_equal(base.cpu().numpy()[mask], before.cpu().numpy()[mask])


def test_pack_input_modulated_channel(shape):
    """Third channel c * a / s when requested; BF16 rounding of the FP32 product."""
    import torch
    from paper_2312_13094_amd import nn
    net = _net(_params(), shape)
    a, b, c = _input(shape, 11)
    a[3] = 0.0
    dv = nn.dense_view(shape)
    scale = torch.zeros(int(nn.lib().nn_rms_scratch_floats()), device="cuda")
    scale[0] = 4.0
    ta, tb, tc = (torch.from_numpy(v).cuda() for v in (a, b, c))
    net.pack_input(ta, dv, tb, dv, tc, dv, scale=scale, c_times_a=True)
    torch.cuda.synchronize()
    x = _from_bits(net.x8, 8, shape)
    ref = N.input_channels(a, b, c, 4.0, c_times_a=True)
    # a/4, b/4 are exact in FP32; the product c * (a/4) rounds once to FP32, then to BF16
    np.testing.assert_array_equal(x[0], N.bf16_round((a / np.float32(4.0)).astype(np.float32)))
    np.testing.assert_array_equal(x[1], N.bf16_round((b / np.float32(4.0)).astype(np.float32)))
    np.testing.assert_array_equal(
        x[2], N.bf16_round((c * (a / np.float32(4.0))).astype(np.float32)))
    assert rel_l2(x[2], ref[2]) <= 5e-3
    assert np.all(x[2][3] == 0.0) and np.all(x[3:] == 0.0)


def test_layer1_from_fields_equals_pack_then_conv(shape):
    """nn_conv_gelu_fields (layer 1 forming its input from three fields, two
    of them read through a padded view) writes bitwise the pre-activations
    and activations of nn_pack_input followed by nn_conv_gelu(1), and so the
    same layer-3 output."""
    import torch
    from paper_2312_13094_amd import nn
    net = _net(_params(), shape)
    a, b, c = _input(shape, 12)
    dv = nn.dense_view(shape)
    nz, ny, nx = shape
    pad = (nz + 4, ny + 4, nx + 9)

    def padded(v):
        P = np.zeros(pad, np.float32)
        P[2:2 + nz, 2:2 + ny, 3:3 + nx] = v
        return torch.from_numpy(P).cuda()

    pv = nn.View(2 * pad[1] * pad[2] + 2 * pad[2] + 3, pad[2], pad[1] * pad[2])
    pa, pb = padded(a), padded(b)
    tc = torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).cuda()
    scale = torch.zeros(int(nn.lib().nn_rms_scratch_floats()), device="cuda")
    scale[0] = 2.7
    net.pack_input(pa, pv, pb, pv, tc, dv, scale=scale, c_times_a=True)
    net.forward(keep=True, ydense=True)
    torch.cuda.synchronize()
    want = [t.clone() for t in (net.z1, net.a1, net.y)]
    for t in (net.z1, net.a1, net.y):
        t.zero_()
    net.forward(keep=True, ydense=True, scale=scale, fields=(pa, pv, pb, pv, tc, dv, True))
    torch.cuda.synchronize()
    for got, w in zip((net.z1, net.a1, net.y), want):
        assert torch.equal(got, w)
    assert float(want[2].abs().max()) > 0


@pytest.mark.parametrize("layer", [1, 2, 3])
def test_weight_gradients_match_oracle(layer, shape):
    import torch
    from paper_2312_13094_amd import nn
    rng = np.random.default_rng(10 + layer)
    cin, gc = {1: (8, 16), 2: (16, 16), 3: (16, 8)}[layer]
    cin_real, co_real = {1: (3, 16), 2: (16, 16), 3: (16, 1)}[layer]
    x = np.zeros((cin,) + shape, np.float32)
    x[:cin_real] = rng.standard_normal((cin_real,) + shape)
    g = np.zeros((gc,) + shape, np.float32)
    g[:co_real] = rng.standard_normal((co_real,) + shape)
    net = _net(_params(), shape)
    xt = torch.from_numpy(_bits(_cl(x))).cuda()
    gt = torch.from_numpy(_bits(_cl(g))).cuda()
    net.grads.zero_()
    nz, ny, nx = shape
    nn._chk(nn.lib().nn_wgrad(layer, nz, ny, nx, nn._p(xt), nn._p(gt), nn._p(net.ws),
                              nn._p(net.grads), 0, nn._s()))
    torch.cuda.synchronize()
    gw, gb = N.conv3d_wgrad(N.bf16_round(x[:cin_real]), N.bf16_round(g[:co_real]))
    first = net.grads.cpu().numpy()
    parts = nn.split_params(first)
    w_got, b_got = parts[2 * layer - 2], parts[2 * layer - 1]
    assert rel_l2(w_got, gw) <= 1e-4
    assert rel_l2(b_got, gb) <= 1e-4
    # accumulate: a second sample's gradient is added with one FP32 rounding
    g2 = np.zeros_like(g)
    g2[:co_real] = rng.standard_normal((co_real,) + shape)
    gt.copy_(torch.from_numpy(_bits(_cl(g2))))
    net.grads.zero_()
    nn._chk(nn.lib().nn_wgrad(layer, nz, ny, nx, nn._p(xt), nn._p(gt), nn._p(net.ws),
                              nn._p(net.grads), 0, nn._s()))
    second = net.grads.cpu().numpy()
    net.grads.copy_(torch.from_numpy(first))
    nn._chk(nn.lib().nn_wgrad(layer, nz, ny, nx, nn._p(xt), nn._p(gt), nn._p(net.ws),
                              nn._p(net.grads), 1, nn._s()))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(net.grads.cpu().numpy(), first + second)


@pytest.mark.parametrize("layer", [2, 3])
def test_data_gradients_match_oracle(layer, shape):
    import torch
    from paper_2312_13094_amd import nn
    rng = np.random.default_rng(20 + layer)
    p = _params(5)
    net = _net(p, shape)
    w = _oracle_params(p)[2 * layer - 2]
    co_real, gcin = (16, 16) if layer == 2 else (1, 8)
    gin = np.zeros((gcin,) + shape, np.float32)
    gin[:co_real] = rng.standard_normal((co_real,) + shape)
    zprev = rng.standard_normal((16,) + shape).astype(np.float32)
    gt = torch.from_numpy(_bits(_cl(gin))).cuda()
    zt = torch.from_numpy(_bits(_cl(zprev))).cuda()
    out = torch.zeros(int(np.prod(shape)) * 16, dtype=torch.int16, device="cuda")
    nz, ny, nx = shape
    nn._chk(nn.lib().nn_dgrad_gelu(layer, nz, ny, nx, nn._p(gt), nn._p(net.packed), nn._p(zt),
                                   nn._p(out), nn._s()))
    torch.cuda.synchronize()
    ref = N.conv3d_dgrad(N.bf16_round(gin[:co_real]), w) * N.gelu_grad(N.bf16_round(zprev))
    assert rel_l2(_from_bits(out, 16, shape), ref) <= 5e-3


def test_mse_and_adam(shape):
    import torch
    from paper_2312_13094_amd import nn
    rng = np.random.default_rng(7)
    net = _net(_params(), shape)
    y = rng.standard_normal(shape).astype(np.float32)
    t = rng.standard_normal(shape).astype(np.float32)
    net.y.copy_(torch.from_numpy(y.ravel()))
    net.loss.zero_()
    nz, ny, nx = shape
    tt = torch.from_numpy(t.ravel()).cuda()
    nn._chk(nn.lib().nn_mse(nz, ny, nx, nn._p(net.y), nn._p(tt), None, 1.0, None,
                            nn._p(net.g8), nn._p(net.loss), nn._s()))
    torch.cuda.synchronize()
    assert abs(net.loss.item() - N.mse(y.astype(np.float64), t)) <= 1e-5 * N.mse(y, t)
    g = _from_bits(net.g8, 8, shape)
    ref = 2 * (y.astype(np.float64) - t) / y.size
    assert rel_l2(g[0], ref) <= 5e-3 and np.all(g[1:] == 0)
    # target scaled by 1 / (gain * s), points of a box excluded
    lo, hi = (0, 4, 5), (6, 13, 20)
    m = N.box_mask(shape, lo, hi)
    scale = torch.zeros(int(nn.lib().nn_rms_scratch_floats()), device="cuda")
    scale[0] = 3.0
    net.loss.zero_()
    nn._chk(nn.lib().nn_mse(nz, ny, nx, nn._p(net.y), nn._p(tt), nn._p(scale), 0.25,
                            nn._bp(nn.box(lo, hi)), nn._p(net.g8), nn._p(net.loss), nn._s()))
    torch.cuda.synchronize()
    tsc = t.astype(np.float64) / 0.75
    want = N.masked_mse(y.astype(np.float64), tsc, m)
    assert abs(net.loss.item() - want) <= 1e-5 * want
    g = _from_bits(net.g8, 8, shape)
    ref = 2 * m * (y.astype(np.float64) - tsc) / y.size
    assert rel_l2(g[0], ref) <= 5e-3 and np.all(g[0][m == 0] == 0)
    # Adam: three steps against the textbook update
    p0 = net.params.cpu().numpy().astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0.copy()
    for step in range(1, 4):
        gr = rng.standard_normal(p0.size)
        net.grads.copy_(torch.from_numpy(gr.astype(np.float32)))
        net.adam(lr=1e-2)
        p, m, v = N.adam_step(p, gr.astype(np.float32).astype(np.float64), m, v, step, lr=1e-2)
    torch.cuda.synchronize()
    assert np.abs(net.params.cpu().numpy() - p).max() <= 1e-5
    # bias-free training: biases and their moments stay as they are
    bias = np.zeros(p0.size, bool)
    bias[1296:1312] = bias[8224:8240] = bias[8672] = True
    net.train_bias = False
    mdev = net.m.cpu().numpy().astype(np.float64)
    vdev = net.v.cpu().numpy().astype(np.float64)
    p = net.params.cpu().numpy().astype(np.float64)
    gr = rng.standard_normal(p0.size)
    net.grads.copy_(torch.from_numpy(gr.astype(np.float32)))
    net.adam(lr=1e-2)
    p, m2, v2 = N.adam_step(p, gr.astype(np.float32).astype(np.float64), mdev, vdev, 4, lr=1e-2,
                            frozen=bias)
    torch.cuda.synchronize()
    got = net.params.cpu().numpy()
    assert np.abs(got - p).max() <= 1e-5
    np.testing.assert_array_equal(net.m.cpu().numpy()[bias], mdev[bias].astype(np.float32))


def test_end_to_end_gradient_and_training(shape):
    """All parameter gradients of the MSE through the three layers agree with
    the FP64 oracle network rounded to BF16 wherever the kernels store BF16
    (pre-activations, activations, dL/dy, dL/dz2, dL/dz1), so that only FP32
    accumulation order separates them (it flips a BF16 rounding at a small
    fraction of points: 5e-3 relative); against the unrounded FP64 network
    they agree within the BF16 storage error (5e-2).  A short Adam run on a
    fixed target reduces the loss."""
    import torch
    from paper_2312_13094_amd import nn
    p = _params(8, scale=0.5)
    net = _net(p, shape)
    a, b, c = _input(shape, 9)
    rng = np.random.default_rng(9)
    t = (0.5 * a + 0.1 * rng.standard_normal(shape)).astype(np.float32)
    dv = nn.dense_view(shape)
    ins = [torch.from_numpy(v).cuda() for v in (a, b, c)]
    net.pack_input(ins[0], dv, ins[1], dv, ins[2], dv)
    tt = torch.from_numpy(t.ravel()).cuda()
    net.loss.zero_()
    net.forward(keep=True)
    net.backward(tt)
    torch.cuda.synchronize()
    x = np.stack([N.bf16_round(v) for v in (a, b, c)])
    got = nn.split_params(net.grads.cpu().numpy())
    onet = N.Net(*_oracle_params(p), store=N.bf16_round)
    oloss, ograds = onet.loss_and_grads(x, t[None].astype(np.float64))
    assert abs(net.loss.item() - oloss) <= 1e-3 * oloss
    for k in range(6):
        assert rel_l2(got[k], ograds[k]) <= 5e-3, k
    floss, fgrads = N.Net(*_oracle_params(p)).loss_and_grads(x, t[None].astype(np.float64))
    assert abs(net.loss.item() - floss) <= 2e-2 * floss
    for k in range(6):
        assert rel_l2(got[k], fgrads[k]) <= 5e-2, k
    losses = []
    for _ in range(60):
        net.loss.zero_()
        net.forward(keep=True)
        net.backward(tt)
        net.adam(lr=3e-3)
        losses.append(net.loss.item())
    assert losses[-1] < 0.5 * losses[0]


def test_rms_and_non_finite_flag(shape):
    """nn_rms over a padded view: sqrt(mean(u^2)) within FP32 summation
    error, the same value on every call, and the flag raised by one NaN."""
    import torch
    from paper_2312_13094_amd import nn
    rng = np.random.default_rng(13)
    nz, ny, nx = shape
    py = nx + 3
    pz = (ny + 3) * py
    off = 1 * pz + 2 * py + 1
    u = torch.from_numpy(rng.standard_normal((nz + 2) * pz).astype(np.float32)).cuda()
    idx = off + np.arange(nz)[:, None, None] * pz + np.arange(ny)[None, :, None] * py + \
        np.arange(nx)[None, None, :]
    vals = u.cpu().numpy()[idx].astype(np.float64)
    net = _net(_params(), shape)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = nn.lib()
    got = []
    for _ in range(2):
        nn._chk(L.nn_rms(nz, ny, nx, nn._p(u), nn.View(off, py, pz), nn._p(net.scale),
                         nn._p(flag), nn._s()))
        torch.cuda.synchronize()
        got.append(net.scale[0].item())
    assert got[0] == got[1]
    assert abs(got[0] - np.sqrt(np.mean(vals ** 2))) <= 1e-6 * got[0]
    assert flag.item() == 0
    u[int(idx[3, 5, 7])] = float("nan")
    nn._chk(L.nn_rms(nz, ny, nx, nn._p(u), nn.View(off, py, pz), nn._p(net.scale),
                     nn._p(flag), nn._s()))
    torch.cuda.synchronize()
    assert flag.item() == 1
