"""Learned coarse-grid correction end to end at a small scale (fine 64^3 so 8,
coarse 32^3 so 4, 4 training and 2 held-out models): training on
solver-generated data lowers the one-step error, the corrected coarse run
beats the plain coarse run against the plain fine solve on held-out models,
the correction leaves the source box and zero fields untouched, and
non-finite weights fall back to the fine solve."""
import numpy as np
import pytest

from paper_2312_13094_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_2312_13094_amd import learned as LC
    cfg = synth.cfg_learned(n_fine=64, nt_fine=240, ntrain=4, ntest=2)
    lc = LC.LearnedCorrector(cfg)
    models = []
    steps = [1, 2, 3, 5] + list(range(8, 118, 6))
    train = lc.make_samples(cfg.train_seeds, steps, models)
    test = lc.make_samples(cfg.test_seeds, steps, models)
    before, base = lc.sample_loss(test, models)
    lc.train(train, models, iters=2000, lr=2e-3, seed=0)
    after, _ = lc.sample_loss(test, models)
    return lc, cfg, models, (before, base, after)


def test_training_lowers_one_step_error(trained):
    _, _, _, (before, base, after) = trained
    assert np.isfinite(after)
    assert after < 0.5 * base, (before, base, after)


def test_correction_beats_plain_coarse_on_held_out_models(trained):
    """Every held-out model: the corrected run completes without the guard
    falling back to the fine solve, and its trace error against the fine
    solve is below the plain coarse run's."""
    from paper_2312_13094_amd import learned as LC
    lc, cfg, _, _ = trained
    rows = []
    for seed in cfg.test_seeds:
        lc.set_model(cfg.velocity(seed))
        ref, _, _ = lc.fine_solve()
        plain, _ = lc.coarse_solve()
        res = lc.learned_solve()
        rows.append((seed, bool(res.fallback), LC.trace_error(plain, ref),
                     LC.trace_error(res.traces, ref)))
    for seed, fell_back, e_plain, e_learned in rows:
        assert not fell_back, rows
        assert e_learned < e_plain, rows


def test_correction_is_zero_on_zero_field_and_inside_source_box(trained):
    """N(0) = 0 (bias-free, velocity channel modulated by the field), and the
    source box keeps the plain coarse values."""
    import torch
    lc, cfg, _, _ = trained
    lc.set_model(cfg.velocity(cfg.test_seeds[0]))
    lc.ca.zero_()
    lc.cb.zero_()
    lc.correct(lc.ca, lc.cb)
    torch.cuda.synchronize()
    assert float(lc.coarse.domain(lc.ca).abs().max()) == 0.0
    # a field with energy everywhere: only the box stays bit-identical
    rng = np.random.default_rng(3)
    nc = cfg.n_coarse
    f = torch.from_numpy(rng.standard_normal((nc,) * 3).astype(np.float32)).cuda()
    lc.coarse.domain(lc.ca).copy_(f)
    lc.coarse.domain(lc.cb).copy_(f * 0.9)
    lc.correct(lc.ca, lc.cb)
    torch.cuda.synchronize()
    out = lc.coarse.domain(lc.ca).cpu().numpy()
    lo, hi = list(lc.skip.lo), list(lc.skip.hi)
    inside = tuple(slice(a, b) for a, b in zip(lo, hi))
    np.testing.assert_array_equal(out[inside], f.cpu().numpy()[inside])
    assert np.abs(out - f.cpu().numpy()).max() > 0.0


def test_graph_replay_equals_eager_run(trained):
    """The captured corrected run replays bit-identically to the eager one,
    for a second model loaded into the same buffers and with eager work
    between the replays."""
    lc, cfg, _, _ = trained
    out = []
    for seed in cfg.test_seeds[:2]:
        lc.set_model(cfg.velocity(seed))
        eager = lc.learned_solve(guard=False)
        g1 = lc.learned_solve(guard=False, graph=True)
        plain, _ = lc.coarse_solve()
        g2 = lc.learned_solve(guard=False, graph=True)
        np.testing.assert_array_equal(g1.traces, eager.traces)
        np.testing.assert_array_equal(g2.traces, eager.traces)
        out.append(eager.traces)
    assert not np.array_equal(out[0], out[1])


def test_non_finite_network_falls_back_to_fine_solve(trained):
    import torch
    lc, cfg, _, _ = trained
    saved = lc.net.params.clone()
    try:
        lc.net.params[100] = float("nan")
        lc.net.pack()
        lc.set_model(cfg.velocity(cfg.test_seeds[0]))
        ref, _, _ = lc.fine_solve()
        res = lc.learned_solve()
        assert res.fallback
        np.testing.assert_array_equal(res.traces, ref)
    finally:
        lc.net.params.copy_(saved)
        lc.net.pack()
        torch.cuda.synchronize()
