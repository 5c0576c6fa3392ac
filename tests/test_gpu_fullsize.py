"""Parity at the benchmark's full size and launch configuration (m = 2,000,000, n = 64,
kappa = 1e12, s1 = 8192, s2 = 256, seed 1), step by step on outputs the oracle can compute
one at a time, and on properties that hold at any size:

  * bucket/sign codes of sampled rows: bit-exact;
  * W1 rows of sampled buckets: 1e-13 relative (oracle sums the bucket's rows exactly);
  * W from the device W1 with the oracle's S2: 1e-13 relative;
  * R0 from the device W with the oracle's Householder: 1e-12 relative;
  * Q0 rows: row-wise backward error |v - x R0| <= 4 n u |x||R0| (Section 5.2);
  * G = Q0^T Q0 (accurately summed Gram of the device Q0): 1e-13 relative; R1^T R1 = G;
  * Q, R: ||I - Q^T Q||_F <= 10 n u, ||V - Q R||_F / ||V||_F <= 10 n u, R against the
    generator's closed form R(diag(sigma) W^T).
"""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import sketch as osk
from oracle.dense import householder_r
from oracle.rand_cholqr import U_PAPER

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")

M, N, KAPPA, S1, S2, SEED = 2_000_000, 64, 1e12, 8192, 256, 1


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gram_accurate(Q, chunk=4096):
    """Q^T Q with short accumulation chains: chunk Grams (K = chunk) added pairwise.  A single
    GEMM over K = 2e6 rows is off by a few 1e-14 relative, more than the orthogonality error."""
    m, n = Q.shape
    pad = (-m) % chunk
    Qp = torch.cat([Q, Q.new_zeros(pad, n)]) if pad else Q
    blocks = Qp.reshape(-1, chunk, n)
    parts = torch.bmm(blocks.transpose(1, 2).contiguous(), blocks)
    while parts.shape[0] > 1:
        if parts.shape[0] % 2:
            parts = torch.cat([parts, torch.zeros_like(parts[:1])])
        parts = parts[0::2] + parts[1::2]
    return parts[0]


@pytest.fixture(scope="module")
def run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("fullsize: generating V", flush=True)
    V, (U, sig, W) = synth.make_V(M, N, KAPPA, SEED, return_factors=True)
    del U
    Vd = torch.from_numpy(V).to("cuda")
    p = rc.Plan(M, N, S1, S2, SEED)
    Q, R = p.factor(Vd)
    it = {k: v.cpu().numpy() for k, v in p.intermediates().items()}
    yield {"V": V, "Vd": Vd, "sig": sig, "W": W, "plan": p, "Q": Q, "R": R, "it": it}
    p.close()


def test_codes_sampled_rows(run):
    p = run["plan"]
    for row0, cnt in [(0, 4096), (M // 2 + 1, 777), (M - 1000, 1000)]:
        b, g = p.sketch_hash(row0, cnt)
        ob, og = osk.countsketch_hash(cnt, S1, SEED, row0=row0)
        np.testing.assert_array_equal(b.cpu().numpy().astype(np.int64), ob)
        np.testing.assert_array_equal(g.cpu().numpy(), og)


def test_w1_sampled_buckets(run):
    V, W1 = run["V"], run["it"]["W1"]
    b, g = osk.countsketch_hash(M, S1, SEED)
    rng = np.random.Generator(np.random.PCG64(0))
    for bk in rng.choice(S1, size=48, replace=False):
        rows = np.flatnonzero(b == bk)
        terms = V[rows] * g[rows, None].astype(np.float64)
        ref = np.array([math.fsum(col) for col in terms.T])
        assert np.linalg.norm(W1[bk] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_w_from_device_w1(run):
    it = run["it"]
    S2m = osk.gaussian_sketch(S2, S1, SEED)
    ref = S2m @ it["W1"]
    assert rel(it["W"], ref) <= 1e-13


def test_r0_from_device_w(run):
    it = run["it"]
    R0o, st, _ = householder_r(it["W"])
    assert st == 0
    assert rel(it["R0"], R0o) <= 1e-12


def test_q0_rows_backward_error_and_gram(run):
    p, Vd, V, it = run["plan"], run["Vd"], run["V"], run["it"]
    Q0a, Q0b = p.q0_twice(Vd)
    torch.cuda.synchronize()
    assert torch.equal(Q0a, Q0b)
    rows = np.random.Generator(np.random.PCG64(1)).choice(M, size=2000, replace=False)
    X = Q0a[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    R0 = it["R0"]
    lhs = np.abs(V[rows] - X @ R0)
    rhs = 4 * N * U_PAPER * (np.abs(X) @ np.abs(R0))
    assert np.all(lhs <= rhs + 1e-300)
    G = gram_accurate(Q0a).cpu().numpy()
    assert rel(np.triu(it["G"]), np.triu(G)) <= 1e-13
    assert rel(it["R1"].T @ it["R1"], G) <= 1e-13


def test_final_q_and_r(run):
    Q, R, Vd = run["Q"], run["R"], run["Vd"]
    n = N
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    orth = torch.linalg.norm(eye - gram_accurate(Q)).item()
    res = (torch.linalg.norm(Vd - Q @ R) / torch.linalg.norm(Vd)).item()
    tgt = 10 * n * U_PAPER
    print(f"fullsize: orth {orth:.3e} res {res:.3e} target {tgt:.3e}", flush=True)
    assert orth <= tgt and res <= tgt
    Rh = R.cpu().numpy()
    A = run["sig"][:, None] * run["W"].T
    Rref = np.linalg.qr(A, mode="r")
    Rref = Rref * np.sign(np.diag(Rref))[:, None]
    assert np.all(np.diag(Rh) > 0) and np.all(np.tril(Rh, -1) == 0)
    assert rel(Rh, Rref) <= 1e-12
