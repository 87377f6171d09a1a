"""Pins of the oracle's Philox4x64-10 (Salmon et al., SC'11).

The oracle's block function is checked against numpy's independent
implementation (``numpy.random.Philox``, 4x64, 10 rounds).  numpy increments
its counter before encrypting, so block ``c`` of the oracle equals the first
four raw words of a numpy generator whose counter is set to ``c - 1``.
"""
import numpy as np
import pytest


def numpy_block(ctr, key):
    c = [int(w) for w in ctr]
    # subtract one with borrow across the four 64-bit words
    val = sum(w << (64 * i) for i, w in enumerate(c))
    val = (val - 1) % (1 << 256)
    words = np.array([(val >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return g.random_raw(4)


CASES = [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [1, 2]),
    ([0, 7, 3, 1], [1, 0]),
    ([199, 255, 7, 1], [1, 0]),
    ([2**64 - 1, 5, 0, 1], [12345, 67890]),
    ([0, 0, 0, 0], [2**64 - 1, 2**64 - 1]),
    ([123456789, 987654321, 42, 0], [3, 511]),
]


@pytest.mark.parametrize("ctr,key", CASES)
def test_philox_matches_numpy(orc, ctr, key):
    got = orc.philox4x64_10(ctr, key)
    exp = numpy_block(ctr, key)
    assert [int(x) for x in got] == [int(x) for x in exp]


def test_philox_random_cases_match_numpy(orc):
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr[0] += 1  # keep the borrow out of the upper words half the time
        assert [int(x) for x in orc.philox4x64_10(ctr, key)] == \
               [int(x) for x in numpy_block(ctr, key)]


def test_u01_range_and_resolution(orc):
    assert orc.u01(0) == 0.0
    assert orc.u01(2**64 - 1) == 1.0 - 2.0**-53
    assert orc.u01(1 << 11) == 2.0**-53
    assert orc.u01((1 << 11) - 1) == 0.0


def test_u01_uniformity_chi_square(orc):
    # 4096 blocks x 4 words -> 16384 uniforms in 64 bins
    vals = []
    for i in range(4096):
        vals.extend(orc.u01(w) for w in orc.philox4x64_10([i, 3, 1, 1], [1, 0]))
    counts, _ = np.histogram(vals, bins=64, range=(0.0, 1.0))
    expected = len(vals) / 64.0
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 63 degrees of freedom: the 99.99% quantile is about 117
    assert chi2 < 117.0
