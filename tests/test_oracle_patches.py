"""Pins for patch extraction, coverage and overlap averaging."""
import itertools

import numpy as np
import pytest

from oracle import patches


@pytest.mark.parametrize("shape,patch,stride,n", [
    ((64, 64), (8, 8), (1, 1), 3249),
    ((512, 512), (10, 10), (1, 1), 253009),
    ((1024, 1024), (10, 10), (1, 1), 1030225),
    ((256, 256, 64), (8, 8, 4), (1, 1, 2), 1922031),
])
def test_patch_counts(shape, patch, stride, n):
    assert int(np.prod(patches.grid_shape(shape, patch, stride))) == n


CASES = [((9,), (3,), (2,)), ((7, 6), (3, 2), (1, 2)), ((5, 6, 7), (2, 3, 2), (1, 1, 2)),
         ((4, 5, 3, 6), (2, 2, 1, 3), (1, 2, 1, 1))]


@pytest.mark.parametrize("shape,patch,stride", CASES)
def test_extract_against_nested_loops(shape, patch, stride):
    rng = np.random.Generator(np.random.PCG64(1))
    img = rng.standard_normal(shape)
    mask = (rng.random(shape) < 0.4).astype(np.uint8)
    X, Mk = patches.extract(img, mask, patch, stride)
    grid = [range(0, m - b + 1, s) for m, b, s in zip(shape, patch, stride)]
    rows = []
    for origin in itertools.product(*grid):
        vals, obs = [], []
        for off in itertools.product(*[range(b) for b in patch]):
            q = tuple(o + f for o, f in zip(origin, off))
            vals.append(img[q])
            obs.append(mask[q] != 0)
        rows.append((vals, obs))
    assert X.shape == (len(rows), int(np.prod(patch)))
    for i, (vals, obs) in enumerate(rows):
        assert np.array_equal(X[i], np.array(vals))
        assert np.array_equal(Mk[i], np.array(obs))


@pytest.mark.parametrize("shape,patch,stride", CASES + [((64, 64), (8, 8), (1, 1))])
def test_coverage_closed_form(shape, patch, stride):
    c = patches.coverage(shape, patch, stride)
    G = patches.grid_shape(shape, patch, stride)
    factors = []
    for m, b, s, g in zip(shape, patch, stride, G):
        q = np.arange(m)
        # number of grid origins j*s (0 <= j < g) with j*s <= q < j*s + b
        lo = np.maximum(0, -(-(q - b + 1) // s))
        hi = np.minimum(g - 1, q // s)
        factors.append(np.maximum(0, hi - lo + 1))
        if s == 1:
            assert np.array_equal(factors[-1], np.minimum.reduce(
                [q + 1, np.full(m, b), m - q, np.full(m, m - b + 1)]))
    expect = factors[0]
    for f in factors[1:]:
        expect = np.multiply.outer(expect, f)
    assert np.array_equal(c, expect)


def test_overlap_average_identity_on_dyadic_image():
    rng = np.random.Generator(np.random.PCG64(2))
    shape, patch, stride = (20, 17), (5, 4), (1, 1)
    img = rng.integers(0, 256, size=shape) / 256.0
    X, _ = patches.extract(img, np.ones(shape, np.uint8), patch, stride)
    out = patches.overlap_average(X, shape, patch, stride)
    assert np.array_equal(out, img)


def test_shape_errors():
    with pytest.raises(patches.ShapeError):
        patches.grid_shape((8, 8), (9, 2), (1, 1))
    with pytest.raises(patches.ShapeError):
        patches.grid_shape((8, 8), (2, 2), (0, 1))
    with pytest.raises(patches.ShapeError):
        patches.grid_shape((2, 2, 2, 2, 2), (1,) * 5, (1,) * 5)
    with pytest.raises(patches.ShapeError):
        patches.check_covered((9,), (3,), (4,))       # pixel 3 and 7,8 uncovered
    patches.check_covered((9,), (3,), (3,))
