"""Pins of the oracle's acquisition policies (oracle/acquire.py) against what
their definitions fix independently of the code: binomial counts, uniform hop
lengths, the reduction of the targeted rule to the uniform one, the expected
count sum(p) = rho M, zero acquisitions where the rule gives p = 0, and
per-pixel frequencies proportional to p over many frames."""
import numpy as np
from scipy import stats

from oracle import acquire

SEED = 0xACC0
SHAPE = (48, 40)
M = SHAPE[0] * SHAPE[1]


def test_uniform_counts_are_binomial_and_frames_differ():
    rho = 0.15
    counts = [int(acquire.uniform_mask(SHAPE, rho, SEED, 3, f).sum()) for f in range(60)]
    # the 60 counts are draws of Binomial(M, rho): Kolmogorov-Smirnov against it
    ks = stats.kstest(counts, stats.binom(M, rho).cdf)
    assert ks.pvalue > 1e-3, ks
    a = acquire.uniform_mask(SHAPE, rho, SEED, 3, 1)
    assert np.array_equal(a, acquire.uniform_mask(SHAPE, rho, SEED, 3, 1))
    assert not np.array_equal(a, acquire.uniform_mask(SHAPE, rho, SEED, 3, 2))
    assert not np.array_equal(a, acquire.uniform_mask(SHAPE, rho, SEED, 4, 1))


def test_uniform_neighbours_are_independent():
    rho = 0.3
    m = np.concatenate([acquire.uniform_mask(SHAPE, rho, SEED, 1, f).ravel() for f in range(20)])
    # 2 x 2 table of (pixel, right neighbour) acquisitions: chi-square test of independence
    a, b = m[:-1].astype(bool), m[1:].astype(bool)
    table = np.array([[np.sum(a & b), np.sum(a & ~b)], [np.sum(~a & b), np.sum(~a & ~b)]])
    assert stats.chi2_contingency(table).pvalue > 1e-3


def test_line_hop_hops_are_uniform_on_one_to_hmax():
    rho = 0.2
    hmax = max(1, int(np.floor(2.0 / rho + 0.5)) - 1)     # 9
    starts, hops = [], []
    for f in range(6):
        m = acquire.line_hop_mask(SHAPE, rho, SEED, 2, f)
        for row in m:
            pos = np.nonzero(row)[0]
            starts.append(pos[0])
            hops.extend(np.diff(pos))
    hops = np.array(hops)
    assert hops.min() >= 1 and hops.max() <= hmax
    assert max(starts) < hmax
    observed = np.bincount(hops, minlength=hmax + 1)[1:]
    assert stats.chisquare(observed).pvalue > 1e-3      # uniform on 1 .. hmax
    m = acquire.line_hop_mask((200, 400), rho, SEED, 0, 0)
    assert abs(m.mean() - 2.0 / (hmax + 1)) < 0.01       # fraction 1 / mean hop


def test_targeted_reduces_to_uniform():
    rho = 0.12
    w = np.full(SHAPE, 3.7)
    u = acquire.uniform_mask(SHAPE, rho, SEED, 5, 9)
    # constant weights: p = rho everywhere, the uniform rule on the same uniforms
    assert np.array_equal(acquire.targeted_mask(w, rho, 0.8, SEED, 5, 9), u)
    # no share for the weights, or no weight at all: the uniform rule again
    rng = np.random.default_rng(1)
    assert np.array_equal(acquire.targeted_mask(rng.random(SHAPE), rho, 0.0, SEED, 5, 9), u)
    assert np.array_equal(acquire.targeted_mask(np.zeros(SHAPE), rho, 0.8, SEED, 5, 9), u)


def test_targeted_expected_count_and_zero_weight_pixels():
    rho, share = 0.1, 0.6
    rng = np.random.default_rng(2)
    w = rng.gamma(2.0, size=SHAPE)
    p = acquire.targeted_probabilities(w, rho, share)
    assert p.max() < 1.0
    assert abs(p.sum() - rho * M) < 1e-9 * M             # closed form: sum p = rho M
    # all of the budget on a band: nothing outside it, p = rho M / |band| inside
    wb = np.zeros(SHAPE)
    wb[10:20, :] = 1.0
    pb = acquire.targeted_probabilities(wb, rho, 1.0).reshape(SHAPE)
    assert np.all(pb[wb == 0] == 0.0)
    assert np.allclose(pb[wb > 0], rho * M / (wb > 0).sum())
    for f in range(5):
        m = acquire.targeted_mask(wb, rho, 1.0, SEED, 0, f)
        assert not m[wb == 0].any()


def test_targeted_frequencies_follow_p():
    rho, share = 0.2, 1.0
    shape = (8, 8)
    w = np.arange(1.0, 65.0).reshape(shape)
    p = acquire.targeted_probabilities(w, rho, share)
    n = 400
    freq = np.sum([acquire.targeted_mask(w, rho, share, SEED, 7, f).ravel() for f in range(n)], axis=0)
    # per pixel a Binomial(n, p_q) count: standardised residuals within 5 sigma, and
    # their sum of squares a chi-square with 64 degrees of freedom
    z = (freq - n * p) / np.sqrt(n * p * (1 - p))
    assert np.all(np.abs(z) < 5)
    assert stats.chi2(64).sf(np.sum(z * z)) > 1e-3
