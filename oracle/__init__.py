"""Plain, slow FP64 CPU oracle for randomized Householder-Cholesky QR with multisketching.

TEST INFRASTRUCTURE ONLY.  This package is the reference that the GPU library is checked
against; it is not part of the product.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the HIP library
(``paper_2309_05868_amd``) and imports nothing from it.

Source: Higgins, Szyld, Boman, Yamazaki, "Analysis of Randomized Householder-Cholesky QR
Factorization with Multisketching" (arXiv 2309.05868).  Notation follows the library: V has
m rows and n columns (the paper writes n rows and m columns), the CountSketch has s1 rows
(paper: p1), the Gaussian sketch s2 rows (paper: p2).

Modules
  philox        Philox4x64-10 counter-based generator (Salmon et al., SC'11), written from its
                published definition; pinned against numpy.random.Philox.
  sketch        the sketch contract: CountSketch bucket/sign per row, Gaussian sketch entries.
  countsketch   W1 = S1 V, correctly rounded per entry (Section 4.2).
  dense         textbook Householder R, Cholesky, row-wise forward substitution, triangular
                product (Algorithms 1-3 steps; Section 5.2 error-analysis subsections).
  rand_cholqr   randQR (Algorithm 1), cholQR (Algorithm 2), rand_cholQR (Algorithm 3),
                cholQR2 (Algorithm 4), shifted CholeskyQR3 (cited in Section 1; parity unpinned),
                and the error measures of Section 6.3.

Every function is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py`` except the
shifted CholeskyQR3 shift constant, which the paper does not state ("parity unpinned").
"""

from . import philox, sketch, countsketch, dense, rand_cholqr  # noqa: F401
from .rand_cholqr import (  # noqa: F401
    U_PAPER,
    rand_cholqr as rand_cholqr_factor,
    rand_qr,
    cholqr,
    cholqr2,
    shifted_cholqr3,
    orth_error,
    residual_error,
    OK,
    E_RANK,
    E_CHOL,
)
