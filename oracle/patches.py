"""N-D overlapping patches: grid, extraction, coverage and overlap averaging.

Test infrastructure, not product code (see ``oracle/__init__.py``).

The paper's N-dimensional inpainting section treats an image of shape
M = (M_0, M_1, ...) cut into patches of shape B with B_d <= M_d in every
dimension.  This module writes that decomposition out plainly:

* along dimension d there are G_d = floor((M_d - B_d) / S_d) + 1 patch origins
  g * S_d, g = 0 .. G_d - 1 (valid patches only, no padding);
* patches are numbered in C order over the grid, pixels of a patch in C order
  over B, so patch i, pixel p sits at image index o_i + b(p);
* the reconstruction averages, at every pixel, the values that all covering
  patches give it.
"""
import itertools

import numpy as np


class ShapeError(ValueError):
    pass


def grid_shape(shape, patch, stride):
    shape, patch, stride = tuple(shape), tuple(patch), tuple(stride)
    if not (1 <= len(shape) <= 4) or len(patch) != len(shape) or len(stride) != len(shape):
        raise ShapeError("ndim must be 1..4 with matching patch and stride")
    for m, b, s in zip(shape, patch, stride):
        if s <= 0 or b <= 0 or b > m:
            raise ShapeError("need 0 < B_d <= M_d and S_d > 0, got M=%s B=%s S=%s"
                             % (shape, patch, stride))
    return tuple((m - b) // s + 1 for m, b, s in zip(shape, patch, stride))


def patch_origins(shape, patch, stride):
    """Image coordinates (N x ndim) of every patch origin, C order over the grid."""
    g = grid_shape(shape, patch, stride)
    axes = [np.arange(gd) * sd for gd, sd in zip(g, stride)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def patch_offsets(patch):
    """Coordinates (P x ndim) of pixel p inside a patch, C order over B."""
    return np.array(list(itertools.product(*[range(b) for b in patch])), dtype=np.int64)


def pixel_index(shape, patch, stride):
    """Linear image index of (patch i, pixel p), an N x P array."""
    org = patch_origins(shape, patch, stride)
    off = patch_offsets(patch)
    coords = org[:, None, :] + off[None, :, :]
    return np.ravel_multi_index(tuple(coords[..., d] for d in range(len(shape))), shape)


def coverage(shape, patch, stride):
    """c(q): number of patches that contain pixel q, by direct counting."""
    idx = pixel_index(shape, patch, stride)
    c = np.zeros(int(np.prod(shape)), dtype=np.int64)
    np.add.at(c, idx.ravel(), 1)
    return c.reshape(shape)


def check_covered(shape, patch, stride):
    if (coverage(shape, patch, stride) == 0).any():
        raise ShapeError("some pixels are covered by no patch")


def extract(image, mask, patch, stride):
    """Masked patch extraction: X[i, p] = y[o_i + b(p)], Mk[i, p] = mask[...] != 0."""
    image = np.asarray(image)
    mask = np.asarray(mask)
    if image.shape != mask.shape:
        raise ShapeError("image and mask shapes differ")
    idx = pixel_index(image.shape, patch, stride)
    X = image.ravel()[idx].astype(np.float64)
    Mk = mask.ravel()[idx] != 0
    return X, Mk


def overlap_average(Y, shape, patch, stride):
    """x_hat(q) = (1 / c(q)) * sum over (i, p) with o_i + b(p) = q of Y[i, p]."""
    idx = pixel_index(shape, patch, stride)
    acc = np.zeros(int(np.prod(shape)), dtype=np.float64)
    np.add.at(acc, idx.ravel(), np.asarray(Y, dtype=np.float64).ravel())
    c = coverage(shape, patch, stride).ravel()
    return (acc / c).reshape(shape)
