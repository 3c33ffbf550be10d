"""Programmatic signal selection (Feature summary: pre-determined indexing
methods, or on-the-fly strategic selections that improve the reconstruction).

Host-side generators of the sampling mask the library takes as input (1 =
the pixel is acquired).  They draw from NumPy's generator seeded by the
caller; the Gibbs sampler's own random numbers are untouched.

* ``uniform_mask``: exactly round(fraction * M) pixels, uniform without
  replacement;
* ``line_hop_mask``: scan lines along the last axis visited by random hops
  (steps uniform on 1 .. 2/fraction - 1, mean 1/fraction), the acquisition
  pattern of a line-hopping scan;
* ``targeted_mask``: weighted sampling without replacement (Efraimidis and
  Spirakis, Inf. Process. Lett. 97(5), 2006: keep the largest u^(1/w)),
  optionally adding to an existing mask -- with the per-pixel posterior
  variance of the reconstruction (``Problem.posterior_variance``) as the
  weights this steers new acquisitions to where the model is least certain.
"""
import numpy as np


def _count(shape, fraction):
    if not 0.0 <= fraction <= 1.0:
        raise ValueError("fraction must lie in [0, 1], got %r" % (fraction,))
    return int(round(fraction * int(np.prod(shape))))


def uniform_mask(shape, fraction, seed):
    """round(fraction * M) pixels chosen uniformly without replacement."""
    shape = tuple(int(s) for s in shape)
    n = _count(shape, fraction)
    rng = np.random.default_rng(seed)
    m = np.zeros(int(np.prod(shape)), np.uint8)
    m[rng.choice(m.size, size=n, replace=False)] = 1
    return m.reshape(shape)


def line_hop_mask(shape, fraction, seed):
    """Every line along the last axis is visited by hops of 1 .. 2/f - 1 pixels
    (uniform, mean 1/f) from a random start; the acquired fraction is f on
    average."""
    shape = tuple(int(s) for s in shape)
    if not 0.0 < fraction <= 1.0:
        raise ValueError("fraction must lie in (0, 1], got %r" % (fraction,))
    rng = np.random.default_rng(seed)
    L = shape[-1]
    lines = int(np.prod(shape[:-1])) if len(shape) > 1 else 1
    hmax = max(1, int(round(2.0 / fraction)) - 1)
    m = np.zeros((lines, L), np.uint8)
    for r in range(lines):
        pos = int(rng.integers(0, hmax))
        while pos < L:
            m[r, pos] = 1
            pos += int(rng.integers(1, hmax + 1))
    return m.reshape(shape)


def targeted_mask(weights, fraction, seed, base=None):
    """A mask with round(fraction * M) acquired pixels in total: the pixels of
    `base` (kept) plus new ones drawn without replacement among the others
    with probability proportional to `weights` (non-negative; pixels of zero
    weight are drawn only when the positive ones run out)."""
    w = np.asarray(weights, np.float64)
    if np.any(~np.isfinite(w)) or np.any(w < 0):
        raise ValueError("weights must be finite and non-negative")
    shape = w.shape
    n = _count(shape, fraction)
    taken = np.zeros(w.size, bool) if base is None else (np.asarray(base).reshape(-1) != 0)
    if taken.size != w.size:
        raise ValueError("base mask shape %s does not match weights %s" % (np.shape(base), shape))
    need = n - int(taken.sum())
    if need < 0:
        raise ValueError("the base mask already holds %d pixels, more than %d" % (taken.sum(), n))
    rng = np.random.default_rng(seed)
    u = rng.random(w.size)
    flat = w.reshape(-1)
    with np.errstate(divide="ignore"):
        # log of the key u^(1/w): larger is preferred; zero weight sorts last
        key = np.where(flat > 0, np.log(u) / np.where(flat > 0, flat, 1.0), -np.inf)
    # zero-weight pixels are ordered among themselves by their uniform
    key2 = np.where(flat > 0, 0.0, u)
    key[taken] = np.nan
    cand = np.nonzero(~taken)[0]
    order = np.lexsort((-key2[cand], -key[cand]))
    out = taken.copy()
    out[cand[order[:need]]] = True
    return out.astype(np.uint8).reshape(shape)
