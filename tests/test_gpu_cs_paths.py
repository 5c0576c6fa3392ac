"""CountSketch parity on the launch paths the full-size configurations take (Algorithm 1 step 1;
Section 4.2: applying S1 adds or subtracts subsets of the rows of V).

  * LDS copies, every wave of a workgroup looping over several 256-row chunks: the workgroup
    count is capped (256 to 1024 partials), so past about 1024 x 256 rows each workgroup owns
    thousands of rows and all four per-wave copies accumulate before their fixed-order sum;
  * bucket index with the scatter's counters in global memory (s1 > 16384; the gather then sorts
    every bucket), which every 128-column configuration with s1 = 2 n^2 = 32768 runs: the hash
    histogram still in LDS up to s1 = 32768, in global memory above;
  * both in FP64 and with the single-precision sketch.

Integer-valued V makes every bucket sum exact in FP64 (and in FP32 while the partial sums stay
below 2^24), so W1 is compared bit for bit with the oracle's correctly rounded sums whatever the
summation order.  At the 16,777,216 x 8 sweep shape (real V), 48 sampled buckets are compared
with math.fsum over the bucket's rows (1e-13 relative).
"""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import sketch as osk
from oracle.countsketch import apply_countsketch

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


def device_w1(V, n, s1, s2, seed, flags=0):
    m = V.shape[0]
    with rc.Plan(m, n, s1, s2, seed=seed, flags=flags) as p:
        Vd = dev(V)
        p.factor(Vd, check=False)
        W1 = p.intermediates()["W1"].cpu().numpy()
        del Vd
    return W1


# (m, n, s1): LDS path with more than 256 rows per workgroup, so every wave loops:
#   2,100,001 x 8, s1 128: 1024 partials of 2304 rows (waves take 3, 2, 2, 2 chunks), ragged last;
#   600,000 x 16, s1 256:  256 partials of 2560 rows;
#   1,000,003 x 32, s1 64: 512 partials of 2048 rows;
#   700,000 x 64, s1 64:   256 partials of 2816 rows.
LDS_CASES = [(2_100_001, 8, 128), (600_000, 16, 256), (1_000_003, 32, 64), (700_000, 64, 64)]
# bucket index with global scatter counters (s1 > 16384): n = 128, 100 and 64 (s1 just above that limit),
# and with the hash histogram in global memory too (s1 > 32768): n = 128 and 64
GLOBAL_CASES = [(100_000, 128, 32_768), (60_000, 100, 20_000), (200_001, 64, 16_385), (150_000, 128, 32_769),
                (120_000, 64, 40_000)]


@pytest.mark.parametrize("m,n,s1", LDS_CASES + GLOBAL_CASES)
def test_w1_integer_bit_exact_fp64(m, n, s1):
    say("countsketch path", m, n, s1)
    s2 = max(n, min(s1, 4 * n))
    V = synth.make_int_V(m, n, seed=m + 7 * n)
    W1 = device_w1(V, n, s1, s2, seed=31)
    b, g = osk.countsketch_hash(m, s1, 31)
    np.testing.assert_array_equal(W1, apply_countsketch(V, b, g, s1))


@pytest.mark.parametrize("m,n,s1", [(2_100_001, 8, 128), (600_000, 16, 256), (100_000, 128, 32_768), (150_000, 128, 32_769)])
def test_w1_integer_bit_exact_fp32_sketch(m, n, s1):
    # |bucket sums| <= rows_per_bucket * bound < 2^24 keeps every FP32 partial sum exact
    say("countsketch path fp32", m, n, s1)
    s2 = max(n, min(s1, 4 * n))
    bound = max(1, min(1000, (2**24 - 1) // (4 * (m // s1 + 64))))
    V = synth.make_int_V(m, n, seed=m + 11 * n, bound=bound)
    W1 = device_w1(V, n, s1, s2, seed=37, flags=rc.FLAG_SKETCH_FP32)
    b, g = osk.countsketch_hash(m, s1, 37)
    np.testing.assert_array_equal(W1, apply_countsketch(V, b, g, s1))


def test_w1_sampled_buckets_sweep_n8():
    # the 16,777,216 x 8 sweep shape (s1 = 2 n^2 = 128, s2 = 4 n = 32): the LDS path with 1024
    # workgroups of 16,384 rows, each wave accumulating 4096 rows into its copy
    m, n, s1, s2, seed = 16_777_216, 8, 128, 32, 208
    say("sweep n=8: generating V")
    V = synth.make_V(m, n, 1e2, seed)
    W1 = device_w1(V, n, s1, s2, seed)
    b, g = osk.countsketch_hash(m, s1, seed)
    order = np.argsort(b, kind="stable")
    starts = np.searchsorted(b[order], np.arange(s1 + 1))
    rng = np.random.Generator(np.random.PCG64(2))
    worst = 0.0
    for bk in rng.choice(s1, size=48, replace=False):
        rows = order[starts[bk]:starts[bk + 1]]
        terms = V[rows] * g[rows, None].astype(np.float64)
        ref = np.array([math.fsum(col) for col in terms.T])
        err = np.linalg.norm(W1[bk] - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err <= 1e-13, (bk, err)
    say(f"sweep n=8: worst sampled bucket error {worst:.2e}")
