"""Batch means of window averages (host statistics of the solver's outputs)."""
import math

import numpy as np
import pytest

from paper_2311_14140_amd import stats


def test_batch_means_of_independent_windows():
    rng = np.random.default_rng(3)
    x = rng.normal(2.0, 0.5, size=(400, 7))
    m, se, lag1 = stats.batch_means(x)
    assert np.allclose(m, x.mean(0))
    assert np.allclose(se, x.std(0, ddof=1) / math.sqrt(400))
    assert np.all(np.abs(lag1) < 4 / math.sqrt(400))


def test_batch_means_flags_correlated_windows():
    """An AR(1) series with coefficient 0.6 shows its lag-1 correlation."""
    rng = np.random.default_rng(4)
    e = rng.normal(size=20000)
    x = np.zeros_like(e)
    for t in range(1, len(e)):
        x[t] = 0.6 * x[t - 1] + e[t]
    _, _, lag1 = stats.batch_means(x)
    assert abs(lag1 - 0.6) < 0.03


def test_window_statistics_of_sample_dicts():
    rng = np.random.default_rng(5)
    wins = [{"n": rng.normal(1, 0.01, 5), "ux": rng.normal(0.1, 0.02, 5), "T": np.ones(5),
             "pxy": rng.normal(size=5), "pxy_mid": rng.normal(size=5), "qx": np.zeros(5),
             "mass_flow": 0.02 + 0.001 * rng.normal(), "n_sampled_steps": 100} for _ in range(30)]
    st = stats.window_statistics(wins)
    assert st["windows"] == 30 and st["steps_per_window"] == 100
    ux = np.array([w["ux"] for w in wins])
    assert np.allclose(st["ux"]["mean"], ux.mean(0))
    assert np.allclose(st["ux"]["se"], ux.std(0, ddof=1) / math.sqrt(30))
    assert np.all(st["T"]["se"] == 0)
    assert st["mass_flow"]["se"] > 0
    with pytest.raises(ValueError):
        stats.window_statistics(wins[:1])
    bad = dict(wins[1], n_sampled_steps=50)
    with pytest.raises(ValueError):
        stats.window_statistics([wins[0], bad])
