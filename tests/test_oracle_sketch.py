"""Pins for the sketch contract and W1 = S1 V (Section 3's CountSketch and Gaussian sketch)."""

import math

import numpy as np
import pytest
from scipy import stats

from oracle import sketch
from oracle.countsketch import apply_countsketch
from oracle.philox import philox4x64_scalar
import synth


def test_hash_matches_scalar_generator():
    m, s1, seed = 37, 1000, 11
    b, g = sketch.countsketch_hash(m, s1, seed, row0=5)
    for i in range(m):
        row = 5 + i
        w = philox4x64_scalar((row // 4, 0, 0, sketch.TAG_COUNTSKETCH), (seed, 0))[row % 4]
        assert b[i] == (w * s1) >> 64
        assert g[i] == (-1 if w & 1 else 1)


def test_bucket_uniform_and_sign_fair():
    # Section 3: the row holding the nonzero and its sign are uniform at random.
    m, s1 = 400_000, 64
    b, g = sketch.countsketch_hash(m, s1, seed=2024)
    assert b.min() >= 0 and b.max() < s1
    counts = np.bincount(b, minlength=s1)
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-3
    plus = int(np.sum(g == 1))
    assert stats.binomtest(plus, m, 0.5).pvalue > 1e-3
    # independence of bucket and sign: sign balance inside each bucket
    t = stats.chi2_contingency(np.stack([np.bincount(b[g == 1], minlength=s1),
                                         np.bincount(b[g == -1], minlength=s1)]))
    assert t.pvalue > 1e-3


def test_bucket_range_large_s1():
    b, _ = sketch.countsketch_hash(10_000, 2**31 - 1, seed=1)
    assert b.min() >= 0 and b.max() < 2**31 - 1
    b, _ = sketch.countsketch_hash(1000, 1, seed=1)
    assert np.all(b == 0)


def test_box_muller_closed_forms():
    u1 = np.array([1.0, math.exp(-0.5), 0.25, 0.25])
    u2 = np.array([0.3, 0.0, 0.25, 0.5])
    z0, z1 = sketch.box_muller(u1, u2)
    assert z0[0] == 0.0 and z1[0] == 0.0                # ln 1 = 0
    assert abs(z0[1] - 1.0) < 1e-15 and z1[1] == 0.0    # r = 1, angle 0
    r = math.sqrt(-2.0 * math.log(0.25))
    assert abs(z0[2]) < 1e-15 * r and abs(z1[2] - r) < 1e-15 * r   # angle pi/2
    assert abs(z0[3] + r) < 1e-15 * r and abs(z1[3]) < 1e-15 * r  # angle pi


def test_uniform_mapping_bounds():
    u1, u2 = sketch.uniforms_from_words(np.array([0, 2**64 - 1], dtype=np.uint64),
                                        np.array([0, 2**64 - 1], dtype=np.uint64))
    assert u1[0] == 2.0 ** -53 and u1[1] == 1.0
    assert u2[0] == 0.0 and u2[1] == 1.0 - 2.0 ** -53


def test_gaussian_sketch_distribution():
    # Section 3: S = G / sqrt(p) with G standard normal.
    s2, s1 = 64, 4096
    S2 = sketch.gaussian_sketch(s2, s1, seed=5)
    assert S2.shape == (s2, s1)
    z = (S2 * math.sqrt(s2)).ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    # rows of different Box-Muller pairs and the two members of a pair are uncorrelated
    c = np.corrcoef(S2[:8])
    assert np.max(np.abs(c - np.eye(8))) < 5 / math.sqrt(s1)


def test_gaussian_sketch_layout_and_ragged_rows():
    s1, seed = 7, 9
    S2 = sketch.gaussian_sketch(6, s1, seed)
    c = sketch.gaussian_scale(6)
    for k in range(s1):
        for blk in range(2):
            y = philox4x64_scalar((k, blk, 0, sketch.TAG_GAUSSIAN), (seed, 0))
            for pair in range(2):
                u1 = ((y[2 * pair] >> 11) + 1) * 2.0 ** -53
                u2 = (y[2 * pair + 1] >> 11) * 2.0 ** -53
                rr = math.sqrt(-2.0 * math.log(u1))
                zs = (rr * math.cos(sketch.TWO_PI * u2), rr * math.sin(sketch.TWO_PI * u2))
                for t in range(2):
                    j = 4 * blk + 2 * pair + t
                    if j < 6:
                        assert S2[j, k] == zs[t] * c
    # a prefix of the rows does not depend on s2 apart from the scale
    S2b = sketch.gaussian_sketch(9, s1, seed)
    np.testing.assert_allclose(S2b[:6] / sketch.gaussian_scale(9), S2 / c, rtol=4e-16, atol=0)


def test_sketches_independent_streams():
    # Proposition of Section 4 needs S1 and S2 drawn independently: different counter tags.
    b, g = sketch.countsketch_hash(4096, 16, seed=77)
    S2 = sketch.gaussian_sketch(4, 4096, seed=77)
    r = stats.pearsonr(g.astype(float), S2[0]).statistic
    assert abs(r) < 5 / math.sqrt(4096)


def test_countsketch_integer_exact_vs_dense():
    # integer-valued V: every sum is exact, so W1 must equal the dense product bit for bit
    V = synth.make_int_V(3000, 7, seed=1)
    b, g = sketch.countsketch_hash(3000, 50, seed=3)
    W1 = apply_countsketch(V, b, g, 50)
    S1 = sketch.countsketch_dense(b, g, 50)
    np.testing.assert_array_equal(W1, S1 @ V)


def test_countsketch_real_vs_dense_and_exact_rounding():
    V = synth.make_V(2000, 5, 1e3, seed=4)
    b, g = sketch.countsketch_hash(2000, 64, seed=8)
    W1 = apply_countsketch(V, b, g, 64)
    S1 = sketch.countsketch_dense(b, g, 64)
    ref = S1 @ V
    assert np.linalg.norm(W1 - ref) <= 1e-14 * np.linalg.norm(ref)
    # correctly rounded: compare one bucket against exact rational arithmetic
    from fractions import Fraction
    rows = np.flatnonzero(b == 3)
    for c in range(5):
        exact = sum(Fraction(float(g[i])) * Fraction(float(V[i, c])) for i in rows)
        assert W1[3, c] == float(exact)


def test_countsketch_empty_buckets_and_empty_input():
    V = np.ones((3, 2))
    W1 = apply_countsketch(V, np.array([0, 0, 0]), np.array([1, -1, 1]), 4)
    np.testing.assert_array_equal(W1, [[1, 1], [0, 0], [0, 0], [0, 0]])
    W1 = apply_countsketch(np.zeros((0, 2)), np.zeros(0, np.int64), np.zeros(0, np.int8), 3)
    assert W1.shape == (3, 2) and not W1.any()


def test_sketched_norms_embed():
    # Proposition of Section 4: ||S2 S1 x|| stays within a constant factor of ||x|| for x in
    # range(V) (checked through the extreme singular values of S2 S1 V versus those of V).
    m, n, s1, s2 = 20000, 8, 128, 32
    V = synth.make_V(m, n, 1.0, seed=12)   # orthonormal columns
    b, g = sketch.countsketch_hash(m, s1, seed=13)
    W = sketch.gaussian_sketch(s2, s1, seed=13) @ apply_countsketch(V, b, g, s1)
    sv = np.linalg.svd(W, compute_uv=False)
    assert 0.2 < sv.min() and sv.max() < 2.5
