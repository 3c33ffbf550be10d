"""Pins for the oracle's Marsaglia-Tsang gamma draws against scipy."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import gamma, philox


@pytest.mark.parametrize("shape", [1.0 / 128, 0.3, 1.0, 2.5, 40.0, 3.0e6])
def test_gamma_draws_follow_gamma_law(shape):
    n = 2500
    lg = np.array([gamma.log_gamma_draw(shape, 777, 1, philox.TAG_GS, c0, 4) for c0 in range(n)])
    if shape < 0.05:
        # the law of ln G is the stable thing to compare for tiny shapes
        g = np.exp(lg.astype(np.float64))
        pv = stats.kstest(g, stats.gamma(shape).cdf).pvalue
    else:
        pv = stats.kstest(np.exp(lg), stats.gamma(shape).cdf).pvalue
    assert pv > 1e-3, pv


def test_gamma_large_shape_moments():
    shape = 1.2e7
    g = np.exp([gamma.log_gamma_draw(shape, 3, 0, philox.TAG_GE, c0, 1) for c0 in range(3000)])
    z = (g.mean() - shape) / (math.sqrt(shape) / math.sqrt(g.size))
    assert abs(z) < 4
    assert abs(g.std() / math.sqrt(shape) - 1) < 0.06


def test_gamma_tiny_shape_stays_finite_in_log_space():
    lg = [gamma.log_gamma_draw(1.0 / 256, 1, 0, philox.TAG_PI_A, c0, 2) for c0 in range(400)]
    assert np.all(np.isfinite(lg))
    assert min(lg) < -700          # would underflow binary64 outside log space


def test_gamma_rejects_bad_shape():
    with pytest.raises(ValueError):
        gamma.log_gamma_draw(0.0, 1, 0, 5, 0, 1)
    with pytest.raises(ValueError):
        gamma.log_gamma_draw(float("nan"), 1, 0, 5, 0, 1)
