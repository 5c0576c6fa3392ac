"""Ragged batches (rcqr_factor_ragged): matrices of one column shape (n, s1, s2) and uneven row
counts factored with every kernel launched once for the batch.  Each member must give bitwise the
Q, R and status of rcqr_factor on a plan of its own shape and seed (its partitions, and so its
summation orders, are those of its own row count), and a sample is compared with the CPU oracle
(R to 1e-10 relative at kappa <= 1e6, 10 n u bounds).  Also: same-shaped batches above 64 columns
and with s2 > 256 (a two-level Householder tree), and the argument checks."""

import numpy as np
import pytest
import torch

import synth
from oracle.rand_cholqr import U_PAPER, rand_cholqr as oracle_rand_cholqr

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


def say(*a):
    print(*a, flush=True)


def solo(V, s1, s2, seed):
    m, n = V.shape
    with rc.Plan(m, n, s1, s2, seed) as p:
        Q, R = p.factor(V, check=False)
        st = p.info()
    return Q, R, st


# (n, s1, s2, row counts): LDS CountSketch (n = 8), bucket index with LDS counters (16, 64),
# 65..128 columns with the global-counter index and a two-level Householder tree (100, 128; the
# 140,001-row member fills the whole Gram grid, the others a part of it)
CLASSES = [
    (8, 128, 32, [5000, 130_001, 64, 20_000]),
    (16, 512, 64, [10_000, 3001, 70_000, 16, 12_345]),
    (64, 8192, 256, [50_000, 20_001, 100, 64]),
    (100, 20_000, 400, [30_000, 7001, 12_000]),
    (128, 32_768, 512, [20_000, 4097, 9000, 140_001]),
]


@pytest.mark.parametrize("n,s1,s2,ms", CLASSES)
def test_ragged_members_equal_solo_calls(n, s1, s2, ms):
    say("ragged", n, s1, s2, ms)
    k = len(ms)
    seeds = [1000 + 17 * b for b in range(k)]
    Vs = [torch.from_numpy(synth.make_V(m, n, 10.0 ** (2 + 3 * (b % 4)), seed=seeds[b])).to("cuda") for b, m in enumerate(ms)]
    Vs[1][:, n // 3] = 0.0  # member 1 is rank deficient: its sketch has a zero pivot
    ref = [solo(V, s1, s2, sd) for V, sd in zip(Vs, seeds)]
    assert ref[1][2][0] == rc.E_RANK
    with rc.Plan(max(ms), n, s1, s2, seed=0, batch=k + 1) as pb:
        for rep in range(2):
            # second repetition: member 2 in place (Q is V), the others into fresh outputs
            Vin = [V.clone() for V in Vs]
            Qs = [None] * k
            if rep == 1:
                Qs[2] = Vin[2]
            Qo, Ro = pb.factor_ragged(Vin, Qs=Qs, seeds=seeds)
            torch.cuda.synchronize()
            st = pb.info_batch(k)
            for b in range(k):
                assert st[b] == ref[b][2], (rep, b)
                if st[b][0] != rc.OK:
                    continue
                assert torch.equal(Qo[b], ref[b][0]) and torch.equal(Ro[b], ref[b][1]), (rep, b)


def test_ragged_members_match_oracle():
    n, s1, s2 = 32, 2048, 128
    ms = [8000, 2500, 15_001]
    seeds = [71, 72, 73]
    Vh = [synth.make_V(m, n, 1e5, seed=sd) for m, sd in zip(ms, seeds)]
    with rc.Plan(max(ms), n, s1, s2, seed=0, batch=3) as pb:
        Qo, Ro = pb.factor_ragged([torch.from_numpy(v).to("cuda") for v in Vh], seeds=seeds)
        torch.cuda.synchronize()
        assert pb.info_batch(3) == [(rc.OK, 0)] * 3
    tgt = 10 * n * U_PAPER
    for b in range(3):
        o = oracle_rand_cholqr(Vh[b], s1, s2, seeds[b])
        assert o["status"] == 0
        Q, R = Qo[b].cpu().numpy(), Ro[b].cpu().numpy()
        assert np.linalg.norm(R - o["R"]) <= 1e-10 * np.linalg.norm(o["R"]), b
        assert np.linalg.norm(Q - o["Q"]) <= 1e-10 * 10 * np.linalg.norm(o["Q"]), b
        assert np.linalg.norm(np.eye(n) - Q.T @ Q) <= tgt
        assert np.linalg.norm(Vh[b] - Q @ R) / np.linalg.norm(Vh[b]) <= tgt


@pytest.mark.parametrize("m,n,s1,s2", [(9000, 100, 4096, 400), (6001, 128, 32_768, 512), (8000, 64, 4096, 300)])
def test_same_shaped_batch_beyond_64_columns_and_256_sketch_rows(m, n, s1, s2):
    say("factor_batch", m, n, s1, s2)
    k, seed = 3, 60
    V = torch.stack([torch.from_numpy(synth.make_V(m, n, 1e9, seed=seed + b)) for b in range(k)]).to("cuda")
    with rc.Plan(m, n, s1, s2, seed=seed, batch=k) as pb:
        Q, R = pb.factor_batch(V)
        torch.cuda.synchronize()
        st = pb.info_batch(k)
    for b in range(k):
        Qs, Rs, sts = solo(V[b], s1, s2, seed + b)
        assert st[b] == sts == (rc.OK, 0)
        assert torch.equal(Q[b], Qs) and torch.equal(R[b], Rs), b


def test_ragged_argument_checks():
    n, s1, s2 = 16, 512, 64
    V = torch.zeros((5000, n), dtype=torch.float64, device="cuda")
    with rc.Plan(4000, n, s1, s2, seed=1, batch=2) as pb:
        with pytest.raises(rc.RcqrError) as e:
            pb.factor_ragged([V])  # more rows than the plan's m
        assert e.value.status == rc.E_INVALID
        with pytest.raises(ValueError):
            pb.factor_ragged([V[:100]] * 3)  # more members than the workspace holds
        with pytest.raises(rc.RcqrError) as e:
            pb.factor_ragged([V[:10]])  # fewer rows than columns
        assert e.value.status == rc.E_INVALID
    with rc.Plan(4000, n, s1, s2, seed=1, batch=1, flags=rc.FLAG_REORTH) as pb:
        with pytest.raises(rc.RcqrError) as e:
            pb.factor_ragged([V[:3000]])
        assert e.value.status == rc.E_UNSUPPORTED
    torch.cuda.synchronize()
