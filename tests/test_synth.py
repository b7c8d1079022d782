"""The seeded input generators: deterministic, well-formed, always terminate."""
import numpy as np
import pytest

from paper_2312_13094_amd import synth


@pytest.mark.parametrize("n", [8, 16, 33, 48, 96, 512])
@pytest.mark.parametrize("seed", [0, 2, 4, 7])
def test_layered_profile(n, seed):
    p = synth.layered_profile(n, seed)
    assert p.shape == (n,) and p.dtype == np.float32
    assert np.all(np.diff(p) >= 0)
    assert p.min() >= 1500.0 and p.max() <= 4500.0
    # every layer at least 4 cells thick
    edges = np.flatnonzero(np.diff(p)) + 1
    th = np.diff(np.concatenate([[0], edges, [n]]))
    assert th.min() >= 4
    np.testing.assert_array_equal(p, synth.layered_profile(n, seed))


def test_headline_layers():
    p = synth.layered_profile(512, 2)
    assert 8 <= len(np.unique(p)) <= 12


def test_ricker_peak_and_delay():
    dt, f0 = 1e-4, 15.0
    q = synth.ricker(2000, dt, f0)
    assert abs(q.max() - 1.0) < 1e-4
    assert abs(np.argmax(q) * dt - 1.0 / f0) < dt


def test_stable_dt_matches_courant():
    assert abs(synth.courant_limit(8, 3) - 0.4529) < 1e-4
    assert abs(synth.courant_limit(4, 2) - 0.6124) < 1e-4
    c = synth.cfg_2d()
    assert abs(c.dt - 2.041e-3) < 1e-6
