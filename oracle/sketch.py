"""The two sketch matrices, generated from one seed.

Section 3 (Preliminaries on Random Sketching) defines both:
  * the CountSketch S1 (s1 x m) has one nonzero per column; the row holding it and its sign
    (+1 or -1) are drawn uniformly at random; it is not rescaled (Section 5.2, remark on the
    norms of an unscaled CountSketch);
  * the Gaussian sketch S2 (s2 x s1) is (1/sqrt(s2)) G with G a dense standard normal matrix.
S1 and S2 are generated independently (Proposition in Section 4).

The paper does not say how the random numbers are produced (Section 6.1 builds S1
explicitly and excludes sketch generation from its timings).  The library and the oracle
share this contract, each implementing it from this description:

  key    = (seed, 0) for Philox4x64-10
  row i of V (column i of S1):  y = Philox((floor(i/4), 0, 0, 1), key), w = y[i mod 4]
      (one generator block serves four consecutive rows)
      bucket h(i) = floor(w * s1 / 2^64)             (high word of the 128-bit product)
      sign   g(i) = -1 if bit 0 of w is set else +1  (the low bit is independent of the
                                                      high bits that pick the bucket)
  entries S2[4b .. 4b+3, k]:     y = Philox((k, b, 0, 2), key)
      two Box-Muller pairs, (y0, y1) -> rows 4b, 4b+1 and (y2, y3) -> rows 4b+2, 4b+3:
      u1 = ((ya >> 11) + 1) * 2^-53  in (0, 1]
      u2 = (yb >> 11) * 2^-53        in [0, 1)
      r = sqrt(-2 ln u1), t = (2 pi) * u2, z_even = r cos t, z_odd = r sin t
      S2[j, k] = z_j * c with c = 1 / sqrt(s2) (each a correctly rounded FP64 operation)
  rows j >= s2 of the last group are discarded.

TEST INFRASTRUCTURE: see the package docstring.
"""

import math

import numpy as np

from .philox import philox4x64, mulhilo64

TAG_COUNTSKETCH = 1
TAG_GAUSSIAN = 2
TWO_PI = 2.0 * math.pi  # the double nearest to 2*pi (doubling math.pi is exact)
_TWO_M53 = 2.0 ** -53


def countsketch_hash(m, s1, seed, row0=0):
    """Bucket h(i) in [0, s1) and sign g(i) in {-1, +1} for rows i = row0 .. row0+m-1."""
    if s1 < 1:
        raise ValueError("s1 must be >= 1")
    rows = np.arange(row0, row0 + m, dtype=np.uint64)
    y = philox4x64(rows >> np.uint64(2), 0, 0, TAG_COUNTSKETCH, seed, 0)
    lane = (rows & np.uint64(3)).astype(np.int64)
    w = np.choose(lane, y) if m else np.zeros(0, dtype=np.uint64)
    hi, _ = mulhilo64(w, np.uint64(s1))
    bucket = hi.astype(np.int64)
    sign = np.where((w & np.uint64(1)) != 0, -1, 1).astype(np.int8)
    return bucket, sign


def uniforms_from_words(ya, yb):
    """Map two 64-bit words to (u1, u2) with u1 in (0, 1] and u2 in [0, 1); exact in FP64."""
    ya = np.asarray(ya, dtype=np.uint64)
    yb = np.asarray(yb, dtype=np.uint64)
    u1 = ((ya >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * _TWO_M53
    u2 = (yb >> np.uint64(11)).astype(np.float64) * _TWO_M53
    return u1, u2


def box_muller(u1, u2):
    """Box-Muller transform: two independent standard normals from two uniforms."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = TWO_PI * u2
    return r * np.cos(t), r * np.sin(t)


def gaussian_scale(s2):
    """c = 1/sqrt(s2): the scaling of Section 3's Gaussian embedding, S = G / sqrt(p)."""
    return 1.0 / math.sqrt(float(s2))


def gaussian_sketch(s2, s1, seed):
    """Dense S2 (s2 x s1, FP64) under the contract in the module docstring."""
    nb = (s2 + 3) // 4
    k = np.arange(s1, dtype=np.uint64)[None, :]
    b = np.arange(nb, dtype=np.uint64)[:, None]
    y0, y1, y2, y3 = philox4x64(k, b, 0, TAG_GAUSSIAN, seed, 0)
    z = np.empty((nb, 4, s1), dtype=np.float64)
    u1, u2 = uniforms_from_words(y0, y1)
    z[:, 0, :], z[:, 1, :] = box_muller(u1, u2)
    u1, u2 = uniforms_from_words(y2, y3)
    z[:, 2, :], z[:, 3, :] = box_muller(u1, u2)
    g = z.reshape(nb * 4, s1)[:s2]
    return g * gaussian_scale(s2)


def countsketch_dense(bucket, sign, s1):
    """S1 as an explicit dense s1 x m matrix (for brute-force checks on tiny inputs only)."""
    m = len(bucket)
    S1 = np.zeros((s1, m), dtype=np.float64)
    S1[np.asarray(bucket), np.arange(m)] = np.asarray(sign, dtype=np.float64)
    return S1
