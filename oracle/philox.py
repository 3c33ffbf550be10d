"""Philox4x32-10 counter-based generator and its uniform / normal transforms.

Test infrastructure, not product code (see ``oracle/__init__.py``).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11, section 3.2): a 4-word
counter and a 2-word key pass through ten rounds; each round multiplies two
counter words by fixed odd constants, keeps both halves of each 64-bit
product, and mixes the high halves with the other two words and the round
key; the key is advanced by a Weyl increment between rounds.

The BPFA paper states nothing about random numbers; the streams below are this
implementation's contract (key/counter layout, 23-bit uniforms, Box-Muller
normals).  The HIP path implements the same contract independently.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

# stream tags (fourth counter word, low byte); the problem id fills the bits above
TAG_ZS = 1      # z/s sweep: (patch, atom pair)
TAG_DICT = 2    # dictionary draw: (pixel position, atom)
TAG_PI_A = 3    # Beta numerator gamma for atom k: (k, attempt)
TAG_PI_B = 4    # Beta denominator gamma for atom k: (k, attempt)
TAG_GS = 5      # weight precision gamma: (0, attempt)
TAG_GE = 6      # noise precision gamma: (0, attempt)
TAG_INIT = 7    # initial dictionary: (pixel position, atom), iteration word 0
TAG_ACQ = 8     # acquisition masks of a served stream: (pixel or line, hop), frame index


def philox4x32_10_int(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on Python integers (one block); same definition."""
    x0, x1, x2, x3 = (int(c) & 0xFFFFFFFF for c in (c0, c1, c2, c3))
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ ka, p1 & 0xFFFFFFFF,
                          (p0 >> 32) ^ x3 ^ kb, p0 & 0xFFFFFFFF)
    return x0, x1, x2, x3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds over broadcastable uint32 counter words.

    Returns four uint32 arrays (the output block).  The key words are scalars.
    """
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    ka = int(k0) & 0xFFFFFFFF
    kb = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = M0 * x0          # exact: both factors < 2^32
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(ka), lo1,
                          hi0 ^ x3 ^ np.uint64(kb), lo0)
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def key_of(seed):
    """Key words from a 64-bit seed: (low 32 bits, high 32 bits)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def block(seed, problem_id, tag, c0, c1, t):
    """Output block for counter (c0, c1, t, tag | problem_id << 8)."""
    k0, k1 = key_of(seed)
    c3 = (int(tag) & 0xFF) | ((int(problem_id) & 0xFFFFFF) << 8)
    return philox4x32_10(c0, c1, t, c3, k0, k1)


def block_int(seed, problem_id, tag, c0, c1, t):
    """Scalar form of block() on Python integers."""
    k0, k1 = key_of(seed)
    c3 = (int(tag) & 0xFF) | ((int(problem_id) & 0xFFFFFF) << 8)
    return philox4x32_10_int(c0, c1, t, c3, k0, k1)


def uniform_int(w):
    """Scalar form of uniform() on a Python integer word."""
    return ((int(w) >> 9) + 0.5) * 2.0 ** -23


def uniform(w):
    """23-bit uniform in (0, 1): (floor(w / 2^9) + 1/2) * 2^-23.

    Every value is a dyadic rational exactly representable in binary32 and
    binary64, so both arithmetic sides see the identical number.
    """
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(ua, ub):
    """Two independent standard normals from two uniforms (Box & Muller 1958).

    Radius sqrt(-2 ln ua) and angle 2*pi*ub; returns (cos branch, sin branch).
    """
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return rad * np.cos(ang), rad * np.sin(ang)
