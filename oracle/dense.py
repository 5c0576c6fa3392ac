"""Textbook dense kernels used by Algorithms 1-4, written as plain loops.

  householder_r         step 2 of Algorithm 1 (hhqr): R factor of a p x n matrix by
                        Householder reflections; only R is needed (Section 5.1).
  cholesky_upper        step 2 of Algorithm 2: G = R^T R with R upper triangular.
  forward_subst_rows    step 3 of Algorithms 1 and 2: X R = B solved row by row by forward
                        substitution (Section 5.2, "Backward Error of the Forward
                        Substitution", which analyses each row of the solve separately).
  triu_product          step 3 of Algorithm 3: R = R1 R0 (Section 4.1 counts it as a
                        matrix multiplication of two triangular factors).

The paper leaves the sign of the Householder diagonal open (LAPACK's dgeqrf is what it
called); the final R of rand_cholQR is required to have a positive diagonal, so
householder_r returns R with a positive diagonal (rows of R multiplied by -1 where needed).

Status codes: OK = 0, E_RANK = 5 (zero or non-finite diagonal of the Householder R),
E_CHOL = 6 (non-positive or non-finite Cholesky pivot); the failing column is 1-based.

TEST INFRASTRUCTURE: see the package docstring.
"""

import math

import numpy as np

OK = 0
E_RANK = 5
E_CHOL = 6


def householder_r(W):
    """R (n x n, upper triangular, positive diagonal) of the Householder QR of W (p x n, p >= n).

    Returns (R, status, column).  Column j's reflector H = I - tau v v^T with v[0] = 1 maps
    x = A[j:, j] to beta e1, beta = -sign(x0) ||x||; it is applied to the trailing columns.
    """
    A = np.array(W, dtype=np.float64, copy=True)
    p, n = A.shape
    if p < n:
        raise ValueError("householder_r needs at least as many rows as columns")
    for j in range(n):
        x = A[j:, j]
        alpha = x[0]
        xnorm = math.sqrt(math.fsum(x[1:] * x[1:])) if p - j > 1 else 0.0
        if xnorm == 0.0:
            continue  # H = I; A[j, j] = alpha already
        beta = -math.copysign(math.hypot(alpha, xnorm), alpha)
        tau = (beta - alpha) / beta
        v = x.copy()
        v[0] = 1.0
        v[1:] = x[1:] / (alpha - beta)
        # Apply H to the trailing columns: A -= tau v (v^T A).
        if j + 1 < n:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= tau * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
    R = np.triu(A[:n, :])
    d = np.diag(R)
    bad = np.flatnonzero(~np.isfinite(d) | (d == 0.0))
    if bad.size:
        return R, E_RANK, int(bad[0]) + 1
    R = R * np.where(d < 0.0, -1.0, 1.0)[:, None]
    return R, OK, 0


def cholesky_upper(G):
    """Upper-triangular R with G = R^T R, column by column; reads the upper triangle of G.

    Returns (R, status, column); a pivot that is not > 0 (including NaN) gives E_CHOL.
    """
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    R = np.zeros((n, n), dtype=np.float64)
    for j in range(n):
        s = G[j, j] - np.dot(R[:j, j], R[:j, j])
        if not (s > 0.0):
            return R, E_CHOL, j + 1
        rjj = math.sqrt(s)
        R[j, j] = rjj
        for c in range(j + 1, n):
            R[j, c] = (G[j, c] - np.dot(R[:j, j], R[:j, c])) / rjj
    return R, OK, 0


def forward_subst_rows(B, R):
    """X with X R = B for upper-triangular R, every row solved by forward substitution.

    Column j of X is (B[:, j] - sum_{k<j} X[:, k] R[k, j]) / R[j, j], with the k-sum taken in
    increasing k (vectorised over rows only).
    """
    B = np.asarray(B, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m, n = B.shape
    X = np.empty_like(B)
    for j in range(n):
        acc = B[:, j].copy()
        for k in range(j):
            acc -= X[:, k] * R[k, j]
        X[:, j] = acc / R[j, j]
    return X


def triu_product(A, B):
    """C = A B for upper-triangular A and B; C[i, j] = sum_{k=i..j} A[i, k] B[k, j]."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    C = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for j in range(i, n):
            C[i, j] = np.dot(A[i, i:j + 1], B[i:j + 1, j])
    return C
