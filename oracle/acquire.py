"""Acquisition masks of a served stream: TEST INFRASTRUCTURE ONLY.

The Feature summary names two ways of choosing which pixels an instrument
measures: pre-determined indexing methods, and on-the-fly strategic
selections that improve the reconstruction.  The paper gives no rule for
either; the three policies below are this implementation's readings, and the
HIP path implements the same rules independently.  Every random number comes
from the Philox contract of ``oracle.philox`` under the server's seed with
the counter (c0, c1, frame index f, TAG_ACQ | stream << 8) and is one 23-bit
uniform u (word 0 of the block); a pixel is acquired when u < p for a
probability p computed in binary64.

* uniform:  every pixel q independently with p = rho (counter (q, 0, f)).
* line hop: each line along the last axis is visited from a random start by
  random hops: with hmax = max(1, floor(2 / rho + 1/2) - 1), the first acquired
  pixel of line r is floor(u_0 hmax) and hop j >= 1 moves floor(u_j hmax) + 1
  pixels on (u_j from counter (r, j, f)); the mean hop is (hmax + 1) / 2,
  about 1 / rho.
* targeted: the stream's last per-pixel posterior variance v (the spread of
  the last samples of its previous frame) steers a share lam of the expected
  acquisitions: p_q = min(1, (1 - lam) rho + lam rho M v_q / sum(v)), with
  p_q = rho everywhere when sum(v) = 0 (counter (q, 0, f)).  The expected
  acquired count is rho M when no p_q is clipped.
"""
import numpy as np

from . import philox


def _uniforms(seed, stream, c0, c1, frame):
    w = philox.block(seed, stream, philox.TAG_ACQ, np.asarray(c0, np.uint64),
                     np.asarray(c1, np.uint64), int(frame))[0]
    return philox.uniform(w)


def uniform_mask(shape, rho, seed, stream, frame):
    M = int(np.prod(shape))
    u = _uniforms(seed, stream, np.arange(M), np.zeros(M), frame)
    return (u < rho).astype(np.uint8).reshape(shape)


def line_hop_mask(shape, rho, seed, stream, frame):
    shape = tuple(int(s) for s in shape)
    L = shape[-1]
    lines = int(np.prod(shape[:-1])) if len(shape) > 1 else 1
    hmax = max(1, int(np.floor(2.0 / rho + 0.5)) - 1)
    m = np.zeros((lines, L), np.uint8)
    for r in range(lines):
        pos = int(np.floor(_uniforms(seed, stream, [r], [0], frame)[0] * hmax))
        j = 1
        while pos < L:
            m[r, pos] = 1
            pos += int(np.floor(_uniforms(seed, stream, [r], [j], frame)[0] * hmax)) + 1
            j += 1
    return m.reshape(shape)


def targeted_probabilities(weights, rho, share):
    v = np.asarray(weights, np.float64).reshape(-1)
    total = float(np.sum(v))
    if not total > 0.0:
        return np.full(v.size, float(rho))
    p = (1.0 - share) * rho + share * rho * v.size * v / total
    return np.minimum(p, 1.0)


def targeted_mask(weights, rho, share, seed, stream, frame):
    shape = np.shape(weights)
    M = int(np.prod(shape))
    p = targeted_probabilities(weights, rho, share)
    u = _uniforms(seed, stream, np.arange(M), np.zeros(M), frame)
    return (u < p).astype(np.uint8).reshape(shape)
