"""Pins of the counter-based generator: the oracle's Philox4x64-10 must equal
numpy's independent implementation, and the range mapping must hit its exact
edge cases and be uniform."""
import numpy as np
import pytest
from scipy import stats

from tests.oracle_util import M64, np_philox, np_uniform_int


@pytest.mark.parametrize("key", [(0, 0), (180108361, 1), (M64, 6), (123456789123, 3)])
def test_philox_matches_numpy(orc, key):
    rng = np.random.default_rng(7)
    ctrs = [(1, 0, 0, 0), (0, 0, 0, 0), (M64, 0, 0, 0), (0, 1, 0, 0), (5, 7, 9, 11), (0, 0, 0, 1)]
    ctrs += [tuple(int(x) for x in rng.integers(0, 1 << 62, size=4)) for _ in range(20)]
    for c in ctrs:
        assert [int(v) for v in orc.philox(c, key)] == np_philox(c, key), (c, key)


def test_uniform_int_edges(orc):
    for n in (1, 2, 3, 7, 256, 76800, 307200, (1 << 32) - 1):
        assert orc.uniform_int(0, n) == 0
        assert orc.uniform_int(M64, n) == n - 1
        assert orc.uniform_int(1 << 63, n) == n // 2
    # agrees with the exact integer formula
    rng = np.random.default_rng(3)
    for _ in range(200):
        u = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        n = int(rng.integers(1, 1 << 40))
        assert orc.uniform_int(u, n) == np_uniform_int(u, n)


def test_uniform_int_chi2(orc):
    n = 10
    counts = np.zeros(n)
    for i in range(20000):
        u = int(orc.philox((i, 0, 0, 0), (99, 4))[0])
        counts[orc.uniform_int(u, n)] += 1
    p = stats.chisquare(counts).pvalue
    assert p > 1e-3, counts
