"""W1 = S1 V for a CountSketch S1 (Section 4.2: applying a CountSketch adds or subtracts
subsets of rows of V).

Row b of W1 is the signed sum of the rows i of V with h(i) = b.  Each entry is returned
correctly rounded (math.fsum over the signed terms), so the oracle's own error is below one
ulp per entry and does not depend on summation order.  The forward-error model of the
paper (Section 5.2, "Forward Error in matrix-matrix multiplication S2 S1 V") bounds any
other summation order by gamma_m |S1||V|.

TEST INFRASTRUCTURE: see the package docstring.
"""

import math

import numpy as np


def apply_countsketch(V, bucket, sign, s1):
    """Return W1 (s1 x n) with W1[b, c] = fl(sum over i with h(i)=b of g(i) V[i, c])."""
    V = np.asarray(V, dtype=np.float64)
    m, n = V.shape
    bucket = np.asarray(bucket, dtype=np.int64)
    sign = np.asarray(sign, dtype=np.float64)
    if bucket.shape != (m,) or sign.shape != (m,):
        raise ValueError("bucket and sign need one entry per row of V")
    W1 = np.zeros((s1, n), dtype=np.float64)
    if m == 0:
        return W1
    order = np.argsort(bucket, kind="stable")
    sorted_b = bucket[order]
    starts = np.flatnonzero(np.r_[True, sorted_b[1:] != sorted_b[:-1]])
    ends = np.r_[starts[1:], m]
    signed = V * sign[:, None]  # exact: multiplying by +-1
    for s, e in zip(starts, ends):
        rows = order[s:e]
        block = signed[rows]
        W1[sorted_b[s]] = [math.fsum(col) for col in block.T]
    return W1
