"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the same seeded inputs.

Tolerances:
  * bucket and sign indices, and W1 of integer-valued V: bit-exact;
  * W1 and W of real V: ||dW||_F / ||W||_F <= 1e-13;
  * R0 and R (kappa <= 1e6): ||dR||_F / ||R||_F <= 1e-10;
  * any kappa: ||I - Q^T Q||_F <= 10 n u and ||V - Q R||_F / ||V||_F <= 10 n u, u = 2^-52;
  * Q0 recomputed by the final pass equals the Gram pass's Q0 bit for bit; two factorizations of
    the same input are bitwise equal.
Sizes span several tiles (64-row waves, 256-row workgroups, 256-row Householder blocks) and
ragged tails.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import sketch as osk
from oracle.countsketch import apply_countsketch
from oracle.dense import householder_r
from oracle.rand_cholqr import U_PAPER, rand_cholqr as oracle_rand_cholqr, shifted_cholqr3 as oracle_scholqr3

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def say(*a):
    print(*a, flush=True)


def lapack_r(A):
    R = np.linalg.qr(A, mode="r")
    return R * np.sign(np.diag(R))[:, None]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


@pytest.mark.parametrize("m,s1,row0", [(1000, 512, 0), (4097, 8192, 3), (333, 1, 0), (257, 2**20 + 7, 10**9)])
def test_hash_bit_exact(m, s1, row0):
    say("hash", m, s1, row0)
    with rc.Plan(max(m, 16), 16, max(s1, 16), 16, seed=1234) as p:
        b, g = p.sketch_hash(row0, m)
        ob, og = osk.countsketch_hash(m, max(s1, 16), 1234, row0=row0)
        np.testing.assert_array_equal(host(b).astype(np.int64), ob)
        np.testing.assert_array_equal(host(g), og)


def test_gaussian_entries_match_oracle():
    s1, s2, seed = 700, 66, 77
    with rc.Plan(1000, 16, s1, s2, seed) as p:
        S = host(p.gaussian_block(0, s2, 0, s1))
        sub = host(p.gaussian_block(5, 7, 690, 10))
    ref = osk.gaussian_sketch(s2, s1, seed)
    # libm-class log/cos/sin differ by an ulp or so between the two sides
    np.testing.assert_allclose(S, ref, rtol=2e-15, atol=2e-15 * np.abs(ref).max())
    np.testing.assert_array_equal(sub, S[5:12, 690:700])


# (m, n, s1): LDS CountSketch (s1 * padded n <= 4096) and bucket-index CountSketch, including
# buckets longer than one sort window (m / s1 > 2048), ragged n and s1 just above the LDS limit.
CS_CASES = [(5000, 8, 128), (10_000, 16, 256), (20_001, 16, 512), (50_000, 64, 8192), (3001, 32, 2048),
            (600_000, 64, 100), (9999, 50, 700), (20_000, 128, 1000), (4321, 100, 333),
            (70_001, 10, 500), (30_000, 32, 256), (20_000, 64, 128), (300_000, 16, 512)]


@pytest.mark.parametrize("m,n,s1", CS_CASES)
def test_countsketch_integer_bit_exact(m, n, s1):
    say("countsketch int", m, n, s1)
    V = synth.make_int_V(m, n, seed=m + n)
    s2 = max(n, 16)
    with rc.Plan(m, n, s1, s2, seed=5) as p:
        p.factor(dev(V), check=False)
        W1 = host(p.intermediates()["W1"])
    b, g = osk.countsketch_hash(m, s1, 5)
    np.testing.assert_array_equal(W1, apply_countsketch(V, b, g, s1))


@pytest.mark.parametrize("m,n,s1,s2,kappa", [(10_000, 16, 512, 64, 1e4), (5000, 8, 128, 32, 1e2), (40_000, 64, 8192, 256, 1e6),
                                              (3001, 32, 2048, 128, 1e3), (9999, 50, 700, 100, 1e5), (777, 10, 40, 20, 1e6),
                                              (20_000, 128, 2048, 512, 1e6), (7000, 100, 1000, 300, 1e5)])
def test_sketches_R0_and_R_match_oracle(m, n, s1, s2, kappa):
    say("rand_cholqr parity", m, n, s1, s2, kappa)
    seed = 11
    V, (U, sig, W) = synth.make_V(m, n, kappa, seed=seed, return_factors=True)
    o = oracle_rand_cholqr(V, s1, s2, seed)
    assert o["status"] == 0
    with rc.Plan(m, n, s1, s2, seed) as p:
        Q, R = p.factor(dev(V))
        it = {k: host(v) for k, v in p.intermediates().items()}
    Q, R = host(Q), host(R)
    assert rel(it["W1"], o["W1"]) <= 1e-13
    assert rel(it["W"], o["W"]) <= 1e-13
    assert rel(it["R0"], o["R0"]) <= 1e-10
    # G and R1 are built from Q0, whose forward error is O(kappa u) (only row-wise backward
    # stability holds, Section 5.2): same kappa scaling as the Q comparison below
    tol_q0 = 1e-10 * max(1.0, kappa / 1e4)
    assert rel(it["R1"], o["R1"]) <= tol_q0
    assert rel(np.triu(it["G"]), np.triu(o["G"])) <= tol_q0
    assert rel(R, o["R"]) <= 1e-10
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    Rref = lapack_r(sig[:, None] * W.T)
    assert rel(R, Rref) <= 1e-10
    assert rel(Q, o["Q"]) <= 1e-10 * max(1.0, kappa / 1e4)
    tgt = 10 * n * U_PAPER
    assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
    assert np.linalg.norm(V - Q @ R) / np.linalg.norm(V) <= tgt


@pytest.mark.parametrize("m,n,s1,s2,kappa", [(10_000, 16, 512, 64, 1e15), (20_000, 64, 8192, 256, 1e12), (30_000, 8, 128, 32, 1e15),
                                              (12_345, 32, 2048, 128, 1e8), (5000, 24, 1152, 96, 1e14),
                                              (30_000, 128, 32768, 512, 1e15), (9000, 72, 10368, 288, 1e12)])
def test_ill_conditioned_bounds(m, n, s1, s2, kappa):
    say("ill conditioned", m, n, s1, s2, kappa)
    V = synth.make_V(m, n, kappa, seed=3)
    with rc.Plan(m, n, s1, s2, seed=3) as p:
        Q, R = p.factor(dev(V))
        R0 = host(p.intermediates()["R0"])
        W = host(p.intermediates()["W"])
    Q, R = host(Q), host(R)
    tgt = 10 * n * U_PAPER
    assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
    assert np.linalg.norm(V - Q @ R) / np.linalg.norm(V) <= tgt
    assert np.all(np.diag(R) > 0)
    # the device Householder R0 of the device W agrees with the oracle's Householder of it
    R0o, st, _ = householder_r(W)
    assert st == 0 and rel(R0, R0o) <= 1e-12


@pytest.mark.parametrize("n", [64, 16, 128])
def test_q0_recompute_is_bitwise_identical_and_runs_are_deterministic(n):
    m, s1, s2 = 30_000, 2 * n * n, 4 * n
    V = dev(synth.make_V(m, n, 1e12, seed=9))
    with rc.Plan(m, n, s1, s2, seed=9) as p:
        Qa, Ra = p.factor(V)
        Qa, Ra = Qa.clone(), Ra.clone()
        Qb, Rb = p.factor(V)
        a, b = p.q0_twice(V)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert torch.equal(Qa, Qb) and torch.equal(Ra, Rb)


def test_in_place_and_strided_rows():
    m, n, s1, s2 = 4000, 16, 512, 64
    V = synth.make_V(m, n, 1e6, seed=21)
    with rc.Plan(m, n, s1, s2, seed=21) as p:
        Qref, Rref = p.factor(dev(V))
        Qref, Rref = host(Qref), host(Rref)
        # in place: Q overwrites V
        Vd = dev(V)
        Q, R = p.factor(Vd, Q=Vd)
        np.testing.assert_array_equal(host(Q), Qref)
        # rows with a leading dimension larger than n (odd, so the unaligned path runs)
        big = torch.zeros((m, n + 3), dtype=torch.float64, device="cuda")
        big[:, :n] = dev(V)
        Q2, R2 = p.factor(big[:, :n])
        np.testing.assert_array_equal(host(R2), Rref)
        np.testing.assert_array_equal(host(Q2), Qref)


def test_failure_statuses():
    m, n, s1, s2 = 3000, 16, 512, 64
    V = synth.make_V(m, n, 1e3, seed=5)
    Vz = V.copy()
    Vz[:, 7] = 0.0
    with rc.Plan(m, n, s1, s2, seed=5) as p:
        p.factor(dev(Vz), check=False)
        assert p.info() == (rc.E_RANK, 8)
        Vn = V.copy()
        Vn[11, 3] = np.nan
        p.factor(dev(Vn), check=False)
        assert p.info()[0] in (rc.E_RANK, rc.E_CHOL)
        # the plan recovers on the next good input
        Q, R = p.factor(dev(V))
        assert p.info() == (rc.OK, 0)
        with pytest.raises(rc.RcqrError):
            p.factor(dev(Vz))


def test_cholqr2_comparator():
    m, n = 20_000, 16
    good = synth.make_V(m, n, 1e4, seed=40)
    with rc.Plan(m, n, 512, 64, seed=40) as p:
        Q, R = p.cholqr2(dev(good))
        Q, R = host(Q), host(R)
        tgt = 10 * n * U_PAPER
        assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
        assert rel(R, lapack_r(good)) <= 1e-10
        hard = synth.make_V(m, n, 1e12, seed=41)
        Q, R = p.cholqr2(dev(hard), check=False)
        st, col = p.info()
        assert st == rc.E_CHOL or np.linalg.norm(np.eye(n) - host(Q).T @ host(Q)) > 1e3 * tgt
        # rand_cholQR on the same plan still succeeds
        Q, R = p.factor(dev(hard))
        assert np.linalg.norm(np.eye(n) - host(Q).T @ host(Q)) <= tgt


@pytest.mark.parametrize("n,s1,s2,k_mid", [(16, 512, 64, 1e10), (64, 8192, 256, 1e9), (100, 20_000, 400, 1e8)])
def test_scholqr3_comparator(n, s1, s2, k_mid):
    m = 20_000 + 37
    tgt = 10 * n * U_PAPER
    with rc.Plan(m, n, s1, s2, seed=50) as p:
        # moderate kappa: R against the oracle's shifted CholeskyQR3 and LAPACK
        say(f"scholqr3: n={n} kappa=1e5")
        V = synth.make_V(m, n, 1e5, seed=50 + n)
        Q, R = p.scholqr3(dev(V))
        Qo, Ro, st, _ = oracle_scholqr3(V)
        assert st == 0
        Q, R = host(Q), host(R)
        assert rel(R, Ro) <= 1e-10 and rel(R, lapack_r(V)) <= 1e-10
        assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
        assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
        # in place (Q aliases V): bitwise the same as out of place
        Vi = dev(V)
        Qi, Ri = p.scholqr3(Vi, Q=Vi)
        np.testing.assert_array_equal(host(Qi), Q)
        np.testing.assert_array_equal(host(Ri), R)
        # inside its range (Section 6.3: up to about 1e11)
        say(f"scholqr3: n={n} kappa={k_mid:.0e}")
        Vm = synth.make_V(m, n, k_mid, seed=60 + n)
        Q, R = p.scholqr3(dev(Vm))
        Q, R = host(Q), host(R)
        assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
        assert np.linalg.norm(Vm - Q @ R) / np.linalg.norm(Vm) <= tgt
        # past it: breaks down or misses the target, while rand_cholQR on the same plan does not
        say(f"scholqr3: n={n} kappa=1e15")
        Vw = synth.make_V(m, n, 1e15, seed=70 + n)
        Q, R = p.scholqr3(dev(Vw), check=False)
        st, _ = p.info()
        assert st == rc.E_CHOL or np.linalg.norm(np.eye(n) - host(Q).T @ host(Q)) > tgt
        Q, R = p.factor(dev(Vw))
        Q = host(Q)
        assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt



# Gram pass grid: one workgroup per 512 rows (eight 64-row tiles), at most 256 -- one, two and
# 256 workgroups and the cap
@pytest.mark.parametrize("m", [64, 511, 512, 513, 131_072, 131_073])
def test_gram_grid_edges(m):
    n, s1, s2 = 16, 512, 64
    say("gram grid", m)
    V = synth.make_V(m, n, 1e4, seed=17)
    with rc.Plan(m, n, s1, s2, seed=17) as p:
        Q, R = p.factor(dev(V))
        G = host(p.intermediates()["G"])
        Q0a, Q0b = p.q0_twice(dev(V))
        Q0 = host(Q0a)
        assert np.array_equal(Q0, host(Q0b))
    Q, R = host(Q), host(R)
    # the device Gram against the Gram of the device Q0, entrywise within m u |Q0|^T |Q0|: a
    # workgroup partial dropped or counted twice would be off by whole tiles
    bound = m * U_PAPER * (np.abs(Q0).T @ np.abs(Q0))
    assert np.all(np.abs(np.triu(G) - np.triu(Q0.T @ Q0)) <= np.triu(bound))
    tgt = 10 * n * U_PAPER
    assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
    assert np.linalg.norm(V - Q @ R) / np.linalg.norm(V) <= tgt
    assert rel(R, lapack_r(V)) <= 1e-10


@pytest.mark.parametrize("m,n,s1,s2", [(50_000, 64, 8192, 256), (20_001, 128, 32_768, 512), (10_000, 8, 128, 32),
                                       (30_000, 32, 2048, 128)])
def test_sketch_at_plan_is_bitwise_the_per_call_sketch(m, n, s1, s2):
    # S1 made once by rcqr_plan (RCQR_FLAG_SKETCH_AT_PLAN) gives bitwise the factorizations of a
    # plan that makes it in every call, over several inputs in a row (the index is reused)
    say("sketch at plan", m, n, s1, s2)
    Vs = [dev(synth.make_V(m, n, k, seed=80 + i)) for i, k in enumerate((1e3, 1e10, 1e14))]
    with rc.Plan(m, n, s1, s2, seed=8) as p0, rc.Plan(m, n, s1, s2, seed=8, flags=rc.FLAG_SKETCH_AT_PLAN) as p1:
        for V in Vs + Vs[:1]:
            Qa, Ra = p0.factor(V)
            Qb, Rb = p1.factor(V)
            torch.cuda.synchronize()
            assert torch.equal(Qa, Qb) and torch.equal(Ra, Rb)
            ia, ib = p0.intermediates(), p1.intermediates()
            assert torch.equal(ia["W1"], ib["W1"])
