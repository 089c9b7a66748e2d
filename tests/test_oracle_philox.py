"""Pins of the oracle's counter-based Gaussian generator (CPU only).

The generator is Philox4x64-10 (Salmon et al., SC 2011) with Box-Muller
normals; numpy ships an independent implementation of the same Philox
variant, which pins the raw words, and scipy's normal CDF pins the
distribution of the normals."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox


def _numpy_words(ctr, key):
    # numpy's Philox advances its 256-bit counter before producing a block,
    # so the block of counter c comes from a generator started at c - 1
    c = ctr[0] + (ctr[1] << 64) + (ctr[2] << 128) + (ctr[3] << 192)
    k = key[0] + (key[1] << 64)
    return [int(w) for w in np.random.Philox(counter=c - 1, key=k).random_raw(4)]


@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 0, 0, 0), (12345, 0)),
                                     ((123456789, 99, 0, 0), (2 ** 64 - 1, 0)),
                                     ((2 ** 63 + 7, 2 ** 40, 3, 2 ** 62), (0xDEADBEEF, 0x1234)),
                                     ((8191, 4095, 0, 0), (0, 0))])
def test_raw_words_equal_numpy_philox(ctr, key):
    mine = philox.philox4x64(tuple(np.uint64(c) for c in ctr), key)
    assert [int(w) for w in mine] == _numpy_words(ctr, key)


def test_vectorized_words_equal_numpy_over_many_counters():
    q = np.arange(1, 2001, dtype=np.uint64)
    w = philox.philox4x64((q, np.uint64(17), np.uint64(0), np.uint64(0)), (99, 0))
    for i in (0, 1, 2, 500, 1998, 1999):
        ref = _numpy_words((int(q[i]), 17, 0, 0), (99, 0))
        assert [int(w[t][i]) for t in range(4)] == ref


def test_uniform_range_endpoints():
    u = philox.uniform53(np.array([0, 2 ** 11 - 1, 2 ** 64 - 1], dtype=np.uint64))
    assert u[0] == 2.0 ** -53 and u[1] == 2.0 ** -53 and u[2] == 1.0


def test_matrix_entries_equal_scalar_route():
    """The vectorized columns equal the entry computed alone with Python
    integers and the math module, including the ragged last row group."""
    n, d, seed = 37, 5, 2024
    R = philox.gaussian_matrix(n, d, seed)
    assert R.flags.f_contiguous and R.shape == (n, d)
    for i in range(n):
        for j in range(d):
            assert R[i, j] == philox.entry(i, j, seed)


def test_columns_are_keyed_not_sequential():
    """Column j depends on (seed, i, j) only: appended blocks equal the
    matching slice of one long draw, and n does not change a column."""
    R = philox.gaussian_matrix(101, 12, 7)
    assert np.array_equal(philox.gaussian_columns(101, 5, 12, 7), R[:, 5:])
    assert np.array_equal(philox.gaussian_matrix(64, 12, 7), R[:64])
    assert not np.array_equal(philox.gaussian_matrix(101, 12, 8), R)


def test_normals_distribution():
    """Kolmogorov-Smirnov against N(0,1), moments, and no correlation
    between the two normals of a Box-Muller pair or between columns."""
    R = philox.gaussian_matrix(40000, 6, 3)
    z = R.ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    pair = np.corrcoef(R[0::2, 0], R[1::2, 0])[0, 1]
    cross = np.corrcoef(R[:, 0], R[:, 1])[0, 1]
    assert abs(pair) < 0.03 and abs(cross) < 0.03
