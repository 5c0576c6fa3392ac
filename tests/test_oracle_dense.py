"""Pins for the oracle's dense steps against closed forms (tests/golden) and LAPACK."""

import os

import numpy as np
import pytest
import scipy.linalg

from oracle import dense


def read_golden(path):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append([float(v) for v in vals])
    return {k: np.array(v) for k, v in out.items()}


def lapack_r(A):
    R = np.linalg.qr(A, mode="r")
    return R * np.sign(np.diag(R))[:, None]


def test_householder_golden(golden_dir):
    g = read_golden(os.path.join(golden_dir, "householder_orthogonal_columns.txt"))
    R, status, _ = dense.householder_r(g["A"])
    assert status == dense.OK
    np.testing.assert_allclose(R, g["R"], rtol=0, atol=4e-16 * 5)


@pytest.mark.parametrize("p,n,seed", [(10, 3, 0), (64, 16, 1), (300, 40, 2), (5, 5, 3)])
def test_householder_vs_lapack(p, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((p, n))
    R, status, _ = dense.householder_r(A)
    assert status == dense.OK
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    Rl = lapack_r(A)
    assert np.linalg.norm(R - Rl) <= 1e-13 * np.linalg.norm(Rl)
    # R^T R = A^T A (Householder QR is a QR of A)
    G = A.T @ A
    assert np.linalg.norm(R.T @ R - G) <= 1e-13 * np.linalg.norm(G)


def test_householder_graded_columns_backward_stable():
    # column-wise backward error of Householder QR (Section 5.2, c = 29 bound)
    rng = np.random.Generator(np.random.PCG64(7))
    A = rng.standard_normal((50, 6)) * np.logspace(0, -12, 6)
    R, status, _ = dense.householder_r(A)
    Rl = lapack_r(A)
    for j in range(6):
        assert np.linalg.norm(R[:, j] - Rl[:, j]) <= 1e-12 * np.linalg.norm(A[:, j])


def test_householder_negative_leading_entry_and_zero_tail():
    A = np.array([[-3.0, 1.0], [0.0, 2.0], [0.0, 0.0]])
    R, status, _ = dense.householder_r(A)
    assert status == dense.OK
    np.testing.assert_allclose(R, [[3.0, -1.0], [0.0, 2.0]], atol=1e-15)


def test_householder_rank_status():
    A = np.array([[1.0, 2.0], [0.0, 0.0], [0.0, 0.0]])  # second column = 2 x first
    _, status, col = dense.householder_r(A)
    assert status == dense.E_RANK and col == 2
    A = np.array([[1.0, 0.0], [np.nan, 1.0]])
    _, status, col = dense.householder_r(A)
    assert status == dense.E_RANK
    _, status, col = dense.householder_r(np.zeros((4, 3)))
    assert status == dense.E_RANK and col == 1


def test_cholesky_golden(golden_dir):
    g = read_golden(os.path.join(golden_dir, "cholesky_2x2.txt"))
    R, status, _ = dense.cholesky_upper(g["G"])
    assert status == dense.OK
    np.testing.assert_array_equal(R, g["R"])


@pytest.mark.parametrize("n,seed", [(1, 0), (8, 1), (33, 2), (64, 3)])
def test_cholesky_vs_lapack(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((3 * n + 2, n))
    G = A.T @ A
    R, status, _ = dense.cholesky_upper(G)
    assert status == dense.OK
    L = np.linalg.cholesky(G)
    assert np.linalg.norm(R - L.T) <= 1e-13 * np.linalg.norm(L)


def test_cholesky_reads_upper_triangle_only():
    rng = np.random.Generator(np.random.PCG64(9))
    A = rng.standard_normal((20, 5))
    G = A.T @ A
    Gu = np.triu(G) + np.tril(np.full((5, 5), 123.0), -1)
    np.testing.assert_array_equal(dense.cholesky_upper(G)[0], dense.cholesky_upper(Gu)[0])


def test_cholesky_breakdown_status():
    G = np.array([[1.0, 2.0], [2.0, 1.0]])  # indefinite
    _, status, col = dense.cholesky_upper(G)
    assert status == dense.E_CHOL and col == 2
    _, status, col = dense.cholesky_upper(np.array([[0.0]]))
    assert status == dense.E_CHOL and col == 1
    _, status, col = dense.cholesky_upper(np.array([[4.0, 0.0], [0.0, np.nan]]))
    assert status == dense.E_CHOL and col == 2


def test_substitution_golden(golden_dir):
    g = read_golden(os.path.join(golden_dir, "substitution_3x3.txt"))
    X = dense.forward_subst_rows(g["B"], g["R"])
    np.testing.assert_array_equal(X, g["X"])


@pytest.mark.parametrize("m,n,seed", [(100, 1, 0), (1000, 16, 1), (257, 64, 2)])
def test_substitution_vs_scipy(m, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    B = rng.standard_normal((m, n))
    X = dense.forward_subst_rows(B, R)
    ref = scipy.linalg.solve_triangular(R, B.T, trans="T", lower=False).T
    assert np.linalg.norm(X - ref) <= 1e-13 * np.linalg.norm(ref)


def test_substitution_rowwise_backward_error():
    # Section 5.2: each row satisfies x (R + dR_i) = v with |dR_i| <= gamma_n |R|, so the
    # row-wise residual |v - x R| is bounded by gamma_n |x| |R|.
    rng = np.random.Generator(np.random.PCG64(5))
    n = 40
    R = np.triu(rng.standard_normal((n, n))) * np.logspace(0, -10, n)[None, :] + np.diag(np.logspace(0, -10, n))
    B = rng.standard_normal((500, n))
    X = dense.forward_subst_rows(B, R)
    u = 2.0 ** -53
    gamma = n * u / (1 - n * u)
    lhs = np.abs(B - X @ R)
    rhs = gamma * (np.abs(X) @ np.abs(R))
    assert np.all(lhs <= 2 * rhs + 1e-300)


def test_triu_product_vs_matmul():
    rng = np.random.Generator(np.random.PCG64(6))
    A = np.triu(rng.standard_normal((9, 9)))
    B = np.triu(rng.standard_normal((9, 9)))
    C = dense.triu_product(A, B)
    assert np.all(np.tril(C, -1) == 0)
    assert np.linalg.norm(C - A @ B) <= 1e-14 * np.linalg.norm(A @ B)
    # the order matters: A B differs from B A for generic triangular factors
    assert np.linalg.norm(C - B @ A) > 1e-3
