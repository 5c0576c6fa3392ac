"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws inputs; it holds none of the factorization's arithmetic.

make_V(m, n, kappa, seed)
    V = U diag(sigma) W^T, U the Q factor of an m x n standard normal matrix, W the Q factor of
    an n x n standard normal matrix (both drawn from one PCG64 stream seeded with `seed`),
    sigma log-spaced from 1 down to 1/kappa.  Section 6.3 builds its test matrices the same
    way (random orthogonal factors around a diagonal of log-equispaced singular values; it
    centres the range on 1, which is only a scaling).
make_int_V(m, n, seed, bound)
    integer-valued FP64 entries in [-bound, bound]; every sum of them is exact in FP64, so a
    CountSketch of it can be compared bit for bit regardless of summation order.
make_requests(count, seed, ...)
    the serving workload: Poisson arrivals, log-uniform m, uniform n, log-uniform kappa.
"""

import math

import numpy as np


def singular_values(n, kappa):
    """sigma_j = kappa^(-j/(n-1)), j = 0..n-1 (sigma_0 = 1, sigma_{n-1} = 1/kappa)."""
    if n == 1:
        return np.ones(1)
    return np.asarray(float(kappa), dtype=np.float64) ** (-np.arange(n) / (n - 1.0))


def make_factors(m, n, kappa, seed):
    """The generator's factors (U, sigma, W) of V = U diag(sigma) W^T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((m, n))
    U, _ = np.linalg.qr(A, mode="reduced")
    del A
    B = rng.standard_normal((n, n))
    W, _ = np.linalg.qr(B)
    return U, singular_values(n, kappa), W


def make_V(m, n, kappa, seed, return_factors=False):
    """Row-major FP64 m x n matrix with 2-norm condition number kappa."""
    U, sigma, W = make_factors(m, n, kappa, seed)
    core = sigma[:, None] * W.T  # diag(sigma) W^T
    V = np.ascontiguousarray(U @ core)
    if return_factors:
        return V, (U, sigma, W)
    return V


def make_int_V(m, n, seed, bound=1000):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(-bound, bound + 1, size=(m, n)).astype(np.float64)


def make_requests(count, seed, rate_per_s=2000.0, m_range=(1e4, 2e6), n_choices=(8, 16, 32, 64, 128),
                  kappa_range=(1e2, 1e15)):
    """Serving workload: list of dicts (arrival_s, m, n, kappa, s1=2n^2, s2=4n, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps)
    lm = rng.uniform(math.log(m_range[0]), math.log(m_range[1]), size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    lk = rng.uniform(math.log(kappa_range[0]), math.log(kappa_range[1]), size=count)
    out = []
    for r in range(count):
        n = int(ns[r])
        out.append({
            "arrival_s": float(arrivals[r]), "m": int(round(math.exp(lm[r]))), "n": n,
            "kappa": float(math.exp(lk[r])), "s1": 2 * n * n, "s2": 4 * n, "seed": 4_000_000 + r,
        })
    return out
