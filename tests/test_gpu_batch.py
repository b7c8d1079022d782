"""Batched multi-shot gradient (uneven apertures, one graph launch) against
per-shot FP64 oracle gradients summed into the full model in shot order."""
import numpy as np
import pytest

import oracle as O
from paper_2312_13094_amd import synth
from gpu_helpers import rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _small_problem(nbl=6):
    return synth.cfg_fwi_batch(n=64, nshots=3, side_lo=4, side_hi=6, unit=8, nt=70, ckpt_every=13,
                               so=8, nbl=nbl, sigma=5.0)


def _oracle_gradient(c, vstart, vtrue):
    full = np.zeros(c.full_shape)
    traces = []
    for s in range(len(c.shapes)):
        sl = tuple(slice(o, o + n) for o, n in zip(c.origins[s], c.shapes[s]))
        g = O.Grid(c.shapes[s], c.spacing, so=c.so, dt=c.dt, nbl=c.nbl, vmax=c.vmax, bc=0)
        q = c.q.astype(np.float64)
        _, _, dobs, _ = O.forward(g, vtrue[sl].astype(np.float64), c.src[s], q, c.rec[s], c.nt)
        v = vstart[sl].astype(np.float64)
        _, _, d, hist = O.forward(g, v, c.src[s], q, c.rec[s], c.nt, history=True)
        _, _, _, gm = O.adjoint(g, v, c.rec[s], d - dobs, c.src[s], c.nt, hist=hist)
        full[sl] += gm
        traces.append((d, dobs))
    vs = vstart.astype(np.float64)
    return full * (-2.0 / vs ** 3), traces


@pytest.mark.parametrize("nbl", [6, 0], ids=["sponge", "no_sponge"])
def test_batch_gradient_matches_per_shot_oracle(nbl):
    import torch
    from paper_2312_13094_amd import fd
    c = _small_problem(nbl)
    vtrue, vstart = c.true_velocity(), c.start_velocity()
    og, traces = _oracle_gradient(c, vstart, vtrue)
    b = fd.Batch(c.spacing, c.so, c.dt, c.vmax, c.nbl, c.shapes, c.origins, c.full_shape, c.nt,
                 c.ckpt_every)
    for s in range(len(c.shapes)):
        b.set_geometry(s, c.src[s], c.rec[s])
    vdev = to_dev(vstart)
    b.set_model(vdev)
    q = [to_dev(c.q) for _ in c.shapes]
    dobs = [to_dev(t[1].astype(np.float32)) for t in traces]
    d = [torch.zeros((c.nt, len(c.rec[s])), device="cuda") for s in range(len(c.shapes))]
    gv = torch.zeros(c.full_shape, device="cuda")
    b.gradient(q, dobs, d, gv)
    torch.cuda.synchronize()
    for s in range(len(c.shapes)):
        assert rel_l2(d[s].double().cpu().numpy(), traces[s][0]) <= 1e-4
    first = gv.cpu().numpy()
    assert rel_l2(first, og) <= 1e-3
    # replays of the captured graph, with eager work in between, are identical
    for _ in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()
        gv.fill_(123.0)
        for t in d:
            t.fill_(-1.0)
        b.gradient(q, dobs, d, gv)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(gv.cpu().numpy(), first)
    b.close()


def test_batch_gradient_independent_of_checkpoint_interval():
    """The gradient and traces are bitwise the same for any checkpoint
    interval: one segment (the forward run stores every imaging factor and
    nothing is recomputed), 13 steps (a partial last segment) and 1 step."""
    import torch
    from paper_2312_13094_amd import fd
    c = _small_problem(6)
    vstart = c.start_velocity()
    rng = np.random.default_rng(4)
    dobs = [to_dev((rng.standard_normal((c.nt, len(c.rec[s]))) * 1e-3).astype(np.float32))
            for s in range(len(c.shapes))]
    q = [to_dev(c.q) for _ in c.shapes]
    out = []
    for k in (c.nt, 13, 1):
        b = fd.Batch(c.spacing, c.so, c.dt, c.vmax, c.nbl, c.shapes, c.origins, c.full_shape,
                     c.nt, k)
        for s in range(len(c.shapes)):
            b.set_geometry(s, c.src[s], c.rec[s])
        b.set_model(to_dev(vstart))
        d = [torch.zeros((c.nt, len(c.rec[s])), device="cuda") for s in range(len(c.shapes))]
        gv = torch.zeros(c.full_shape, device="cuda")
        b.gradient(q, dobs, d, gv)
        torch.cuda.synchronize()
        out.append((gv.cpu().numpy(), [t.cpu().numpy() for t in d]))
        b.close()
    assert np.abs(out[0][0]).max() > 0
    for g, d in out[1:]:
        np.testing.assert_array_equal(g, out[0][0])
        for a_, b_ in zip(d, out[0][1]):
            np.testing.assert_array_equal(a_, b_)


def test_batch_tiles_agree():
    import torch
    from paper_2312_13094_amd import fd
    c = _small_problem()
    vstart = c.start_velocity()
    out = []
    for tile in [(4, 4, 64, 1), (4, 2, 7, 0), (8, 2, 16, 1), (8, 2, 64, 12), (4, 4, 5, 8),
                 (8, 2, 64, 28), (4, 2, 9, 29)]:
        b = fd.Batch(c.spacing, c.so, c.dt, c.vmax, c.nbl, c.shapes, c.origins, c.full_shape,
                     c.nt, c.ckpt_every)
        b.set_tile(*tile)
        for s in range(len(c.shapes)):
            b.set_geometry(s, c.src[s], c.rec[s])
        b.set_model(to_dev(vstart))
        q = [to_dev(c.q) for _ in c.shapes]
        dobs = [torch.zeros((c.nt, len(c.rec[s])), device="cuda") for s in range(len(c.shapes))]
        d = [torch.zeros_like(x) for x in dobs]
        gv = torch.zeros(c.full_shape, device="cuda")
        b.gradient(q, dobs, d, gv)
        torch.cuda.synchronize()
        out.append(gv.cpu().numpy())
        b.close()
    for o in out[1:]:
        np.testing.assert_array_equal(out[0], o)


def test_batch_rejects_aperture_outside_model():
    from paper_2312_13094_amd import fd
    with pytest.raises(fd.FdError):
        fd.Batch((10.0,) * 3, 8, 5e-4, 4500.0, 4, [(32, 32, 32)], [(40, 0, 0)], (64, 64, 64),
                 10, 5)


def test_batch_autotune_matches_oracle_and_cache_reuses_tile(tmp_path):
    """fd_batch_autotune times candidate tiles on the batch's own apertures
    and applies the fastest; the tuned gradient still matches the per-shot
    FP64 oracle.  A second batch of the same apertures takes the tile from
    the JSON cache without timing (ms 0) and gives a bit-identical
    gradient."""
    import json
    import torch
    from paper_2312_13094_amd import fd
    c = _small_problem()
    vtrue, vstart = c.true_velocity(), c.start_velocity()
    og, traces = _oracle_gradient(c, vstart, vtrue)
    cache = str(tmp_path / "batch_tiles.json")
    grads, tiles = [], []
    for run in range(2):
        b = fd.Batch(c.spacing, c.so, c.dt, c.vmax, c.nbl, c.shapes, c.origins, c.full_shape,
                     c.nt, c.ckpt_every)
        for s in range(len(c.shapes)):
            b.set_geometry(s, c.src[s], c.rec[s])
        b.set_model(to_dev(vstart))
        tile, ms = b.autotune(cache)
        assert (ms > 0.0) == (run == 0)
        assert b.tile == tuple(tile)
        tiles.append(tuple(tile))
        q = [to_dev(c.q) for _ in c.shapes]
        dobs = [to_dev(t[1].astype(np.float32)) for t in traces]
        d = [torch.zeros((c.nt, len(c.rec[s])), device="cuda") for s in range(len(c.shapes))]
        gv = torch.zeros(c.full_shape, device="cuda")
        b.gradient(q, dobs, d, gv)
        torch.cuda.synchronize()
        grads.append(gv.cpu().numpy())
        b.close()
    assert tiles[0] == tiles[1]
    with open(cache) as f:
        entries = json.load(f)
    assert len(entries) == 1 and "|batch|8|3|" in next(iter(entries))
    assert rel_l2(grads[0], og) <= 1e-3
    np.testing.assert_array_equal(grads[1], grads[0])
