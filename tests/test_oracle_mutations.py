"""Planted mistakes in the oracle (CPU only) must each be caught by an independent pin.

Each check below compares the oracle with something outside it (numpy's Philox, LAPACK,
SciPy, a dense brute-force product, the generator's closed form).  The test runs the check on
the real oracle (must pass) and on a copy with one plausible mistake patched in (must fail).
"""

import math

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import dense, philox, rand_cholqr as rc, sketch
from oracle import countsketch as cs


def lapack_r(A):
    R = np.linalg.qr(A, mode="r")
    return R * np.sign(np.diag(R))[:, None]


def check_philox():
    bg = np.random.Philox(counter=np.array([0, 3, 0, 1], dtype=np.uint64), key=np.array([9, 0], dtype=np.uint64))
    assert philox.philox4x64_scalar((1, 3, 0, 1), (9, 0)) == tuple(int(x) for x in bg.random_raw(4))


def check_countsketch():
    V = synth.make_int_V(500, 4, seed=2)
    b, g = sketch.countsketch_hash(500, 16, seed=3)
    np.testing.assert_array_equal(cs.apply_countsketch(V, b, g, 16), sketch.countsketch_dense(b, g, 16) @ V)


def check_gaussian_scale():
    S2 = sketch.gaussian_sketch(32, 2048, seed=1)
    var = float(np.var(S2))
    assert abs(var * 32 - 1.0) < 0.05


def check_householder():
    A = np.random.Generator(np.random.PCG64(1)).standard_normal((30, 7))
    R, _, _ = dense.householder_r(A)
    Rl = lapack_r(A)
    assert np.linalg.norm(R - Rl) <= 1e-13 * np.linalg.norm(Rl)


def check_cholesky():
    A = np.random.Generator(np.random.PCG64(2)).standard_normal((30, 7))
    G = A.T @ A
    R, _, _ = dense.cholesky_upper(G)
    assert np.linalg.norm(R - np.linalg.cholesky(G).T) <= 1e-13 * np.linalg.norm(G)


def check_substitution():
    rng = np.random.Generator(np.random.PCG64(3))
    R = np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6)
    B = rng.standard_normal((40, 6))
    ref = scipy.linalg.solve_triangular(R, B.T, trans="T", lower=False).T
    assert np.linalg.norm(dense.forward_subst_rows(B, R) - ref) <= 1e-13 * np.linalg.norm(ref)


def check_rand_cholqr():
    V, (U, sig, W) = synth.make_V(3000, 6, 1e6, seed=4, return_factors=True)
    o = rc.rand_cholqr(V, 72, 24, seed=4)
    Rref = lapack_r(sig[:, None] * W.T)
    assert o["status"] == rc.OK
    assert np.linalg.norm(o["R"] - Rref) <= 1e-10 * np.linalg.norm(Rref)
    assert rc.orth_error(o["Q"]) <= 10 * 6 * rc.U_PAPER


def check_cholqr2_and_scholqr3_r():
    # the comparators' R against LAPACK's R of V (the thin QR is unique; kappa 1e4 keeps both
    # inside their range): a product taken in the wrong order is off by O(kappa^2 u) relative
    V = synth.make_V(2000, 6, 1e4, seed=5)
    Rl = lapack_r(V)
    for fn in (rc.cholqr2, rc.shifted_cholqr3):
        Q, R, st, _ = fn(V)
        assert st == rc.OK
        assert np.linalg.norm(R - Rl) <= 1e-11 * np.linalg.norm(Rl)
        assert rc.orth_error(Q) <= 10 * 6 * rc.U_PAPER


def _philox_no_key_bump(counter, key, rounds=philox.ROUNDS):
    c0, c1, c2, c3 = (int(x) for x in counter)
    k0, k1 = (int(x) for x in key)
    for _ in range(rounds):
        p0, p1 = philox.PHILOX_M0 * c0, philox.PHILOX_M1 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & philox.MASK64, (p0 >> 64) ^ c3 ^ k1, p0 & philox.MASK64
    return c0, c1, c2, c3


def _countsketch_unsigned(V, bucket, sign, s1):
    return cs.__dict__["_orig_apply"](V, bucket, np.ones_like(sign), s1)


def _householder_wrong_tau(W):
    A = np.array(W, dtype=np.float64)
    p, n = A.shape
    for j in range(n):
        x = A[j:, j]
        alpha, xnorm = x[0], float(np.linalg.norm(x[1:]))
        if xnorm == 0.0:
            continue
        beta = -math.copysign(math.hypot(alpha, xnorm), alpha)
        tau = (beta - alpha) / alpha  # mistake: divides by alpha instead of beta
        v = x.copy()
        v[0] = 1.0
        v[1:] = x[1:] / (alpha - beta)
        A[j:, j + 1:] -= tau * np.outer(v, v @ A[j:, j + 1:])
        A[j, j] = beta
        A[j + 1:, j] = 0.0
    R = np.triu(A[:n])
    return R * np.where(np.diag(R) < 0, -1.0, 1.0)[:, None], dense.OK, 0


def _cholesky_no_offdiag_update(G):
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    R = np.zeros((n, n))
    for j in range(n):
        R[j, j] = math.sqrt(G[j, j] - np.dot(R[:j, j], R[:j, j]))
        for c in range(j + 1, n):
            R[j, c] = G[j, c] / R[j, j]  # mistake: drops the sum over earlier rows
    return R, dense.OK, 0


def _subst_transposed(B, R):
    return dense.__dict__["_orig_subst"](B, np.asarray(R).T.copy() + np.triu(R))


def _product_wrong_order(A, B):
    return dense.__dict__["_orig_triu"](B, A)


def _gaussian_unscaled(s2):
    return 1.0


MUTATIONS = [
    ("philox key schedule not bumped", philox, "philox4x64_scalar", _philox_no_key_bump, check_philox),
    ("countsketch sign dropped", cs, "apply_countsketch", _countsketch_unsigned, check_countsketch),
    ("gaussian sketch not scaled by 1/sqrt(s2)", sketch, "gaussian_scale", _gaussian_unscaled, check_gaussian_scale),
    ("householder tau divides by alpha", dense, "householder_r", _householder_wrong_tau, check_householder),
    ("cholesky drops off-diagonal update", dense, "cholesky_upper", _cholesky_no_offdiag_update, check_cholesky),
    ("substitution reads a transposed operand", dense, "forward_subst_rows", _subst_transposed, check_substitution),
    ("comparators' R = R_first R_second", rc, "triu_product", _product_wrong_order, check_cholqr2_and_scholqr3_r),
]

E2E_MUTATIONS = [
    ("R = R0 R1 instead of R1 R0", rc, "triu_product", _product_wrong_order),
    ("householder tau divides by alpha", rc, "householder_r", _householder_wrong_tau),
    # (a CountSketch without signs is still a sketch, and the final Q, R do not depend on the
    # sketch: only the W1 pin above can see that mistake)
    ("cholesky drops off-diagonal update", rc, "cholesky_upper", _cholesky_no_offdiag_update),
]


@pytest.fixture(autouse=True)
def _originals(monkeypatch):
    monkeypatch.setitem(cs.__dict__, "_orig_apply", cs.apply_countsketch)
    monkeypatch.setitem(dense.__dict__, "_orig_subst", dense.forward_subst_rows)
    monkeypatch.setitem(dense.__dict__, "_orig_triu", dense.triu_product)


@pytest.mark.parametrize("name,mod,attr,bad,check", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_unit_pin_catches_mutation(name, mod, attr, bad, check, monkeypatch):
    check()
    monkeypatch.setattr(mod, attr, bad)
    with pytest.raises(AssertionError):
        check()


@pytest.mark.parametrize("name,mod,attr,bad", E2E_MUTATIONS, ids=[m[0] for m in E2E_MUTATIONS])
def test_end_to_end_pin_catches_mutation(name, mod, attr, bad, monkeypatch):
    check_rand_cholqr()
    monkeypatch.setattr(mod, attr, bad)
    with pytest.raises((AssertionError, ValueError, FloatingPointError)):
        check_rand_cholqr()
