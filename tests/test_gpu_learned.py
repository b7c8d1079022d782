"""Learned coarse-grid correction end to end at a small scale (fine 64^3 so 8,
coarse 32^3 so 4): training on solver-generated data lowers the one-step
error, the corrected coarse run beats the plain coarse run against the plain
fine solve on held-out models, and non-finite weights fall back to the fine
solve."""
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
    lc.train(train, models, iters=600, lr=2e-3, seed=0)
    after, _ = lc.sample_loss(test, models)
    return lc, cfg, models, (before, base, after)


def test_training_lowers_one_step_error(trained):
    _, _, _, (before, base, after) = trained
    assert np.isfinite(after)
    assert after < 0.5 * base, (before, base, after)


def test_correction_beats_plain_coarse_on_held_out_models(trained):
    from paper_2312_13094_amd import learned as LC
    lc, cfg, _, _ = trained
    gains, fell_back = [], 0
    for seed in cfg.test_seeds:
        lc.set_model(cfg.velocity(seed))
        ref, _, _ = lc.fine_solve()
        plain, _ = lc.coarse_solve()
        res = lc.learned_solve()
        if res.fallback:          # the guard fired: the fine solve was returned
            np.testing.assert_array_equal(res.traces, ref)
            fell_back += 1
            continue
        gains.append((LC.trace_error(plain, ref), LC.trace_error(res.traces, ref)))
    assert gains, "every held-out run fell back to the fine solve"
    for e_plain, e_learned in gains:
        assert e_learned < e_plain, (gains, fell_back)


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
