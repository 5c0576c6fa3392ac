"""Algorithms 1-4 of the paper, composed from the oracle's plain steps, plus error measures.

  rand_qr        Algorithm 1 (randQR): W = S2 S1 V; R0 = hhqr(W); Q0 = V R0^{-1}.
  cholqr         Algorithm 2 (cholQR): G = V^T V; R = chol(G); Q = V R^{-1}.
  rand_cholqr    Algorithm 3 (rand_cholQR): [Q0, R0] = randQR; [Q, R1] = cholQR(Q0); R = R1 R0.
  cholqr2        Algorithm 4 (cholQR2).
  shifted_cholqr3  shifted CholeskyQR followed by cholQR2 (sCholQR3, cited in Section 1 as
                 stable up to kappa ~ 1/u).  The paper gives no shift; this uses
                 s = 11 (m n + n (n + 1)) u ||V||_F^2 (Fukaya, Kannan, Nakatsukasa, Yamamoto,
                 Yanagisawa, SISC 2020, with ||V||_2 bounded by ||V||_F).  PARITY UNPINNED:
                 only the qualitative behaviour of Section 6.3 (it fails past kappa ~ 1e12)
                 is checked.
  orth_error     ||I - Q^T Q||_F and residual_error ||V - Q R||_F / ||V||_F, the two measures
                 of Section 6.3.

U_PAPER = 2^-52 is the unit roundoff as the paper states it (Section 6.1).

TEST INFRASTRUCTURE: see the package docstring.
"""

import numpy as np

from .countsketch import apply_countsketch
from .dense import E_CHOL, E_RANK, OK, cholesky_upper, forward_subst_rows, householder_r, triu_product
from .sketch import countsketch_hash, gaussian_sketch

U_PAPER = 2.0 ** -52

__all__ = [
    "U_PAPER", "OK", "E_RANK", "E_CHOL", "rand_qr", "cholqr", "rand_cholqr", "cholqr2",
    "shifted_cholqr3", "orth_error", "residual_error",
]


def rand_qr(V, bucket, sign, s1, S2):
    """Algorithm 1 with explicit sketch data; returns a dict of every intermediate."""
    V = np.asarray(V, dtype=np.float64)
    W1 = apply_countsketch(V, bucket, sign, s1)          # step 1, first sketch
    W = np.asarray(S2, dtype=np.float64) @ W1            # step 1, second sketch (a GEMM)
    R0, status, col = householder_r(W)                   # step 2
    out = {"W1": W1, "W": W, "R0": R0, "status": status, "column": col}
    if status != OK:
        out["Q0"] = None
        return out
    out["Q0"] = forward_subst_rows(V, R0)                 # step 3, row-wise substitution
    return out


def cholqr(V):
    """Algorithm 2; returns (Q, R, status, column)."""
    V = np.asarray(V, dtype=np.float64)
    G = V.T @ V                                           # step 1
    R, status, col = cholesky_upper(G)                    # step 2
    if status != OK:
        return None, R, status, col
    return forward_subst_rows(V, R), R, OK, 0             # step 3


def rand_cholqr(V, s1, s2, seed, sketch=None):
    """Algorithm 3.  `sketch` may supply (bucket, sign, S2) to replace the seeded sketch.

    Returns a dict with Q, R, status, column and the intermediates bucket, sign, W1, W, R0,
    Q0, G, R1.
    """
    V = np.asarray(V, dtype=np.float64)
    m, n = V.shape
    if sketch is None:
        bucket, sign = countsketch_hash(m, s1, seed)
        S2 = gaussian_sketch(s2, s1, seed)
    else:
        bucket, sign, S2 = sketch
    out = {"bucket": bucket, "sign": sign}
    rq = rand_qr(V, bucket, sign, s1, S2)                 # step 1
    out.update(rq)
    out.update({"G": None, "R1": None, "Q": None, "R": None})
    if rq["status"] != OK:
        return out
    Q0 = rq["Q0"]
    G = Q0.T @ Q0                                         # step 2: cholQR(Q0) ...
    out["G"] = G
    R1, status, col = cholesky_upper(G)
    out["R1"] = R1
    if status != OK:
        out["status"], out["column"] = status, col
        return out
    out["Q"] = forward_subst_rows(Q0, R1)                 # ... Q = Q0 R1^{-1}
    out["R"] = triu_product(R1, rq["R0"])                 # step 3: R = R1 R0
    return out


def cholqr2(V):
    """Algorithm 4; returns (Q, R, status, column)."""
    Q0, R0, status, col = cholqr(V)
    if status != OK:
        return None, None, status, col
    Q, R1, status, col = cholqr(Q0)
    if status != OK:
        return None, None, status, col
    return Q, triu_product(R1, R0), OK, 0


def shifted_cholqr3(V, shift=None):
    """Shifted CholeskyQR, then cholQR2 on its Q; returns (Q, R, status, column)."""
    V = np.asarray(V, dtype=np.float64)
    m, n = V.shape
    if shift is None:
        fro2 = float(np.sum(V * V))
        shift = 11.0 * (m * n + n * (n + 1)) * U_PAPER * fro2
    G = V.T @ V + shift * np.eye(n)
    Ra, status, col = cholesky_upper(G)
    if status != OK:
        return None, None, status, col
    Qa = forward_subst_rows(V, Ra)
    Q, Rb, status, col = cholqr2(Qa)
    if status != OK:
        return None, None, status, col
    return Q, triu_product(Rb, Ra), OK, 0


def orth_error(Q):
    """||I - Q^T Q||_F (Section 6.3)."""
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[1]
    return float(np.linalg.norm(np.eye(n) - Q.T @ Q, "fro"))


def residual_error(V, Q, R):
    """||V - Q R||_F / ||V||_F (Section 6.3)."""
    V = np.asarray(V, dtype=np.float64)
    return float(np.linalg.norm(V - Q @ R, "fro") / np.linalg.norm(V, "fro"))
