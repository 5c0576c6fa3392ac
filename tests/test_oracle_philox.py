"""Pins for the oracle's Philox4x64-10 against numpy.random.Philox (independent implementation).

numpy's bit generator increments its counter before producing each 4-word block, so the
first block it returns for counter c is the block for c + 1.
"""

import numpy as np
import pytest

from oracle.philox import MASK64, philox4x64, philox4x64_scalar, mulhilo64


def numpy_blocks(counter, key, count):
    bg = np.random.Philox(counter=np.array(counter, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    raw = bg.random_raw(4 * count)
    return [tuple(int(x) for x in raw[4 * i:4 * i + 4]) for i in range(count)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 7, 9, 11), (123, 456)),
    ((2**64 - 3, 1, 0, 2), (2**63 + 17, 99)),
    ((123456789, 0, 0, 1), (42, 0)),
])
def test_scalar_matches_numpy(counter, key):
    blocks = numpy_blocks(counter, key, 3)
    for i, blk in enumerate(blocks):
        c = list(counter)
        c0 = c[0] + i + 1
        carry = c0 >> 64
        c[0] = c0 & MASK64
        c[1] = (c[1] + carry) & MASK64
        assert philox4x64_scalar(c, key) == blk


def test_vectorised_matches_scalar():
    rng = np.random.Generator(np.random.PCG64(3))
    c = rng.integers(0, 2**63, size=(4, 200), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    key = (0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF)
    out = philox4x64(c[0], c[1], c[2], c[3], *key)
    for i in range(200):
        ref = philox4x64_scalar([int(c[j, i]) for j in range(4)], key)
        assert tuple(int(o[i]) for o in out) == ref


def test_mulhilo_exact():
    rng = np.random.Generator(np.random.PCG64(4))
    a = rng.integers(0, 2**64 - 1, size=500, dtype=np.uint64, endpoint=True)
    b = rng.integers(0, 2**64 - 1, size=500, dtype=np.uint64, endpoint=True)
    hi, lo = mulhilo64(a, b)
    for i in range(500):
        p = int(a[i]) * int(b[i])
        assert int(hi[i]) == p >> 64 and int(lo[i]) == p & MASK64
    hi, lo = mulhilo64(np.uint64(MASK64), np.uint64(MASK64))
    assert int(hi) == MASK64 - 1 and int(lo) == 1
