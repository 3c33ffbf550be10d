"""Mask generators of the programmatic signal selection (host side)."""
import numpy as np
import pytest

from paper_2311_15061_amd import sampling


def test_uniform_mask_exact_count_and_seeded():
    m = sampling.uniform_mask((37, 41), 0.1, seed=3)
    assert m.dtype == np.uint8 and m.shape == (37, 41)
    assert m.sum() == round(0.1 * 37 * 41)
    assert np.array_equal(m, sampling.uniform_mask((37, 41), 0.1, seed=3))
    assert not np.array_equal(m, sampling.uniform_mask((37, 41), 0.1, seed=4))


@pytest.mark.parametrize("fraction", [0.05, 0.1, 0.25])
def test_line_hop_mask_fraction_and_gaps(fraction):
    m = sampling.line_hop_mask((128, 256), fraction, seed=1)
    assert abs(m.mean() / fraction - 1) < 0.1
    gaps = np.concatenate([np.diff(np.nonzero(row)[0]) for row in m])
    hmax = int(round(2 / fraction)) - 1
    assert gaps.min() >= 1 and gaps.max() <= hmax          # hops stay within 1 .. 2/f - 1
    assert abs(gaps.mean() * fraction - 1) < 0.1             # mean hop 1/f


def test_targeted_mask_keeps_base_and_prefers_weight():
    rng = np.random.default_rng(0)
    shape = (64, 64)
    base = sampling.uniform_mask(shape, 0.05, seed=7)
    w = np.ones(shape)
    w[:, 32:] = 9.0                                          # the right half 9x as likely
    m = sampling.targeted_mask(w, 0.25, seed=11, base=base)
    assert m.sum() == round(0.25 * 64 * 64)
    assert np.all(m[base != 0] == 1)
    new = (m != 0) & (base == 0)
    right = new[:, 32:].sum() / new.sum()
    assert 0.75 < right < 0.95                               # weighted draw without replacement
    # zero weight is never drawn while positive weight is left
    w0 = np.zeros(shape)
    w0[rng.random(shape) < 0.5] = 1.0
    m0 = sampling.targeted_mask(w0, 0.2, seed=2)
    assert np.all(w0[m0 != 0] > 0)
    assert np.array_equal(m0, sampling.targeted_mask(w0, 0.2, seed=2))


def test_targeted_mask_errors():
    with pytest.raises(ValueError):
        sampling.targeted_mask(-np.ones((4, 4)), 0.5, seed=0)
    with pytest.raises(ValueError):
        sampling.targeted_mask(np.ones((4, 4)), 0.1, seed=0, base=np.ones((4, 4)))
    with pytest.raises(ValueError):
        sampling.uniform_mask((4, 4), 1.5, seed=0)
