"""Philox4x64-10, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11 (the Philox-4x64 round function, multipliers and Weyl key increments).

The paper (Section 6.1) only says the sketches were constructed explicitly and that their
generation time was excluded; it fixes no generator.  The library and this oracle agree on
one counter-based generator so that the sketch every side uses is the same matrix.

TEST INFRASTRUCTURE: see the package docstring.  Pinned in tests/test_oracle_philox.py against
numpy.random.Philox (an independent third-party implementation of the same generator).
"""

import numpy as np

MASK64 = (1 << 64) - 1
# Round multipliers and key increments of Philox-4x64 (Salmon et al., Table 2 / Section 4).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1
ROUNDS = 10


def philox4x64_scalar(counter, key, rounds=ROUNDS):
    """One Philox4x64 block on Python integers: counter (4 words), key (2 words) -> 4 words.

    A round multiplies words 0 and 2 by the two constants (128-bit products), and outputs
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the Weyl constants before
    every round but the first.
    """
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 128-bit product of uint64 arrays a and b, as (hi, lo) uint64 arrays.

    Built from 32x32->64-bit partial products so nothing overflows a uint64.
    """
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | ((mid & _M32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox4x64 over arrays of counters (broadcast); returns four uint64 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & MASK64
    k1 = int(k1) & MASK64
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        hi0, lo0 = mulhilo64(c0, m0)
        hi1, lo1 = mulhilo64(c2, m1)
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return c0, c1, c2, c3
