"""Pins of the oracle's counter-based generator against numpy's independent
Philox4x64-10 and against the definitions of the two derived draws."""
import numpy as np
import pytest
from scipy import stats


def _numpy_block(key, ctr):
    # numpy's Philox increments its 256-bit counter before producing a block,
    # so the block for counter c is the first one produced from counter c - 1.
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array(words, dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((0, 1), (0, 0, 0, 0)),
    ((12345, 2), (17, 3, 0, 0)),
    ((2**64 - 1, 3), (2**64 - 1, 2**64 - 1, 5, 0)),
    ((0xDEADBEEF, 2), (4_799_999, 5, 4095, 0)),
])
def test_philox_known_answers(orc, key, ctr):
    assert np.array_equal(orc.philox_block(ctr, key), _numpy_block(key, ctr))


def test_uniform_and_index_definitions(orc):
    # U = (w >> 11) * 2^-53 and Index(n) = floor(w * n / 2^64), with w word 0
    # of the block keyed (seed, tag) at counter (a, b, inst, 0).
    rng = np.random.default_rng(1)
    for _ in range(200):
        seed, tag = int(rng.integers(0, 2**63)), int(rng.integers(1, 4))
        a, b, inst = int(rng.integers(0, 2**40)), int(rng.integers(0, 64)), int(rng.integers(0, 5000))
        n = int(rng.integers(1, 2**40))
        w = int(_numpy_block((seed, tag), (a, b, inst, 0))[0])
        assert orc.uniform(seed, tag, a, b, inst) == (w >> 11) * 2.0 ** -53
        assert orc.index(seed, tag, a, b, inst, n) == (w * n) >> 64
        assert 0 <= orc.index(seed, tag, a, b, inst, n) < n


def test_first_center_uniform(orc):
    # Algorithm 2 step 1: uniform over the n points (chi-square over seeds).
    n, S = 7, 35000
    counts = np.bincount([orc.first_center(n, s, 0) for s in range(S)], minlength=n)
    assert stats.chisquare(counts).pvalue > 1e-4
