"""Closed-form quantities the paper states, used by tests as pins on the oracle.

  multisketch_embedding  Proposition of Section 4: eps_L = e1 + e2 - e1 e2,
                         eps_H = e1 + e2 + e1 e2, d = d1 + d2 - d1 d2.
  cond_randqr_bound      Theorem "Conditioning of randQR" (Section 5.3):
                         kappa(Q0) <= 33 / (25 sqrt((1 - eps_L)/(1 + eps_H)) - 3).
  orth_bound_rand_cholqr Theorem "rand_cholQR Errors" (Section 5.3):
                         ||Q^T Q - I||_2 <= 5445 / (25 sqrt(.) - 3)^2 (m n + n (n + 1)) u,
                         written with m rows and n columns.
  paper_sketch_sizes     Section 6.2's multisketch sizes: s1 = ceil(8.24 (n^2 + n)) for the
                         CountSketch (eps1 = 0.9, d1 = 0.15) and s2 = ceil(74.3 ln s1) for the
                         Gaussian sketch (eps2 = 0.49); "log" read as the natural logarithm.

TEST INFRASTRUCTURE: see the package docstring.
"""

import math

from .rand_cholqr import U_PAPER


def multisketch_embedding(eps1, eps2, d1, d2):
    return eps1 + eps2 - eps1 * eps2, eps1 + eps2 + eps1 * eps2, d1 + d2 - d1 * d2


def _core(eps_l, eps_h):
    c = 25.0 * math.sqrt((1.0 - eps_l) / (1.0 + eps_h)) - 3.0
    if c <= 0:
        raise ValueError("embedding parameters outside the theorem's range")
    return c


def cond_randqr_bound(eps_l, eps_h):
    return 33.0 / _core(eps_l, eps_h)


def orth_bound_rand_cholqr(eps_l, eps_h, m, n, u=U_PAPER):
    return 5445.0 / _core(eps_l, eps_h) ** 2 * (m * n + n * (n + 1)) * u


def paper_sketch_sizes(n):
    s1 = math.ceil(8.24 * (n * n + n))
    return s1, math.ceil(74.3 * math.log(s1))
