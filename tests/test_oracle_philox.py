"""Pins for the oracle's Philox4x32-10 and its uniform / normal transforms."""
import os

import numpy as np
from scipy import stats

from oracle import philox


def read_kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_known_answer_vectors(golden_dir):
    rows = read_kat(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(v) for v in out] == r[6:10]


def test_vectorised_equals_scalar():
    c0 = np.arange(50, dtype=np.uint64)
    vec = philox.philox4x32_10(c0, 7, 3, 0x105, 0xDEADBEEF, 0x12345678)
    for i in range(50):
        one = philox.philox4x32_10(i, 7, 3, 0x105, 0xDEADBEEF, 0x12345678)
        assert [int(v[i]) for v in vec] == [int(v) for v in one]


def test_uniform_is_exact_dyadic_in_open_interval():
    w = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = philox.uniform(w)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -24
    assert u[3] == 1.5 * 2.0 ** -23
    assert u[4] == 1.0 - 2.0 ** -24
    assert u[5] == 0.5 + 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_uniform_and_normals_distribution():
    w = philox.block(99, 3, philox.TAG_ZS, np.arange(200000, dtype=np.uint64), 5, 17)
    u = philox.uniform(w[0])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    n_cos, n_sin = philox.box_muller(philox.uniform(w[2]), philox.uniform(w[3]))
    assert stats.kstest(n_cos, "norm").pvalue > 1e-3
    assert stats.kstest(n_sin, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(n_cos, n_sin)[0, 1]) < 0.01
    # different words / tags / counters are not correlated
    assert abs(np.corrcoef(philox.uniform(w[0]), philox.uniform(w[1]))[0, 1]) < 0.01


def test_key_and_counter_layout():
    k0, k1 = philox.key_of(0x0123456789ABCDEF)
    assert (k0, k1) == (0x89ABCDEF, 0x01234567)
    a = philox.block(5, 2, philox.TAG_DICT, 3, 4, 9)
    b = philox.philox4x32_10(3, 4, 9, philox.TAG_DICT | (2 << 8), 5, 0)
    assert [int(x) for x in a] == [int(x) for x in b]


def test_integer_path_matches_array_path(golden_dir):
    for r in read_kat(golden_dir):
        assert list(philox.philox4x32_10_int(*r[:6])) == r[6:10]
    for c0 in (0, 1, 12345, 0xFFFFFFFF):
        a = philox.block(0xABCDEF0123, 7, philox.TAG_PI_B, c0, 3, 11)
        b = philox.block_int(0xABCDEF0123, 7, philox.TAG_PI_B, c0, 3, 11)
        assert [int(v) for v in a] == list(b)
        assert philox.uniform_int(b[1]) == float(philox.uniform(a[1]))
