"""nn_wgrad_noalloc (static device scratch, no allocation) against nn_wgrad
(caller workspace): two calls in a row, the second on a smaller volume, each
bit-identical to the workspace entry point and within FP32 accumulation of
the FP64 oracle on the same BF16 operands."""
import numpy as np
import pytest

from oracle import nn as N
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def _bits(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16).view(np.int16)


def _cl(a):
    return np.ascontiguousarray(np.moveaxis(np.asarray(a), 0, -1)).ravel()


def _case(shape, layer, seed):
    rng = np.random.default_rng(seed)
    cin, gc = {1: (8, 16), 2: (16, 16), 3: (16, 8)}[layer]
    cin_real, co_real = {1: (3, 16), 2: (16, 16), 3: (16, 1)}[layer]
    x = np.zeros((cin,) + shape, np.float32)
    x[:cin_real] = rng.standard_normal((cin_real,) + shape)
    g = np.zeros((gc,) + shape, np.float32)
    g[:co_real] = rng.standard_normal((co_real,) + shape)
    return x, g, cin_real, co_real


@pytest.mark.parametrize("layer", [2, 1, 3])
def test_noalloc_wgrad_matches_workspace_entry_point(layer):
    import torch
    from paper_2312_13094_amd import nn
    L = nn.lib()
    # the larger volume needs every persistent block (612 tiles of 32 x 4 x 4);
    # the second call is smaller and leaves most of the scratch as the first
    # call wrote it
    for k, shape in enumerate([(48, 68, 70), (11, 13, 37)]):
        x, g, cin_real, co_real = _case(shape, layer, 40 + 7 * layer + k)
        xt = torch.from_numpy(_bits(_cl(x))).cuda()
        gt = torch.from_numpy(_bits(_cl(g))).cuda()
        nz, ny, nx = shape
        ws = torch.zeros(int(L.nn_wgrad_workspace_bytes(nz, ny, nx)) // 4, device="cuda")
        np_ = int(L.nn_param_count())
        seed = torch.from_numpy(np.random.default_rng(k).standard_normal(np_).astype(np.float32))
        for acc in (0, 1):
            ref = seed.clone().cuda()
            got = seed.clone().cuda()
            nn._chk(L.nn_wgrad(layer, nz, ny, nx, nn._p(xt), nn._p(gt), nn._p(ws), nn._p(ref),
                               acc, nn._s()))
            nn._chk(L.nn_wgrad_noalloc(layer, nz, ny, nx, nn._p(xt), nn._p(gt), nn._p(got), acc,
                                       nn._s()))
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
        gw, gb = N.conv3d_wgrad(N.bf16_round(x[:cin_real]), N.bf16_round(g[:co_real]))
        parts = nn.split_params(got.cpu().numpy() - seed.numpy())
        assert rel_l2(parts[2 * layer - 2], gw) <= 1e-4
        assert rel_l2(parts[2 * layer - 1], gb) <= 1e-4


def test_noalloc_wgrad_rejects_bad_arguments():
    import torch
    from paper_2312_13094_amd import fd, nn
    L = nn.lib()
    x = torch.zeros(16 * 8, dtype=torch.int16, device="cuda")
    grads = torch.zeros(int(L.nn_param_count()), device="cuda")
    assert L.nn_wgrad_noalloc(4, 2, 2, 2, nn._p(x), nn._p(x), nn._p(grads), 0, nn._s()) == \
        fd.FD_EINVAL
    assert L.nn_wgrad_noalloc(1, 0, 2, 2, nn._p(x), nn._p(x), nn._p(grads), 0, nn._s()) == \
        fd.FD_EINVAL
    assert L.nn_wgrad_noalloc(1, 2, 2, 2, None, nn._p(x), nn._p(grads), 0, nn._s()) == \
        fd.FD_EINVAL
