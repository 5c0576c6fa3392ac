"""Batches (rcqr_batch_*): several factorizations of different shapes, each captured as a HIP
graph and launched concurrently on its own stream.  Every replay gives, for every member,
bitwise the Q and R of an eager call on that member's plan, with eager work on the same plans
and streams between replays."""

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")

SHAPES = [(10_000, 16, 512, 64, 1e4), (5000, 8, 128, 32, 1e8), (30_000, 64, 8192, 256, 1e12), (20_001, 50, 5000, 200, 1e6),
          (12_345, 32, 2048, 128, 1e10), (20_000, 128, 32768, 512, 1e8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


def _members(shapes, seed0):
    plans, Vs, V2s = [], [], []
    for i, (m, n, s1, s2, kappa) in enumerate(shapes):
        st = torch.cuda.Stream()
        plans.append(rc.Plan(m, n, s1, s2, seed=seed0 + i, stream=st))
        Vs.append(torch.from_numpy(synth.make_V(m, n, kappa, seed=seed0 + i)).to("cuda"))
        V2s.append(torch.from_numpy(synth.make_V(m, n, 1e3, seed=seed0 + 100 + i)).to("cuda"))
    torch.cuda.synchronize()
    return plans, Vs, V2s


@pytest.mark.parametrize("method", ["rand_cholqr", "cholqr2"])
def test_batch_replays_match_eager(method):
    print("batch:", method, flush=True)
    shapes = SHAPES if method == "rand_cholqr" else [(s[0], s[1], s[2], s[3], 1e4) for s in SHAPES[:4]]
    plans, Vs, V2s = _members(shapes, 40)
    eager = {"rand_cholqr": "factor"}.get(method, method)
    ref = []
    for p, V in zip(plans, Vs):
        with torch.cuda.stream(p.stream):
            Q, R = getattr(p, eager)(V)
        p.stream.synchronize()
        ref.append((Q.clone(), R.clone()))
    b = rc.Batch(plans, Vs, method=method)
    for rep in range(3):
        for Q, R in zip(b.Qs, b.Rs):
            Q.fill_(float("nan"))
            R.fill_(float("nan"))
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        for i, (p, Q, R) in enumerate(zip(plans, b.Qs, b.Rs)):
            assert p.info() == (rc.OK, 0), (rep, i)
            assert torch.equal(Q, ref[i][0]) and torch.equal(R, ref[i][1]), (rep, i)
        # eager work on the same plans (same workspaces and streams) between replays
        for p, V2 in zip(plans, V2s):
            with torch.cuda.stream(p.stream):
                getattr(p, eager)(V2)
        torch.cuda.synchronize()
    b.close()
    for p in plans:
        p.close()
    torch.cuda.synchronize()


def test_batch_refuses_a_repeated_plan():
    plans, Vs, _ = _members(SHAPES[:2], 60)
    with pytest.raises(rc.RcqrError):
        rc.Batch([plans[0], plans[1], plans[0]], [Vs[0], Vs[1], Vs[0]])
    for p in plans:
        p.close()
    torch.cuda.synchronize()


# rcqr_factor_batch: same-shaped members in one set of launches (LDS and bucket-index
# CountSketch, 8 to 64 columns, ragged m)
@pytest.mark.parametrize("m,n,s1,s2", [(10_000, 16, 512, 64), (5000, 8, 128, 32), (20_001, 50, 5000, 200), (30_000, 64, 8192, 256),
                                       (3001, 32, 2048, 128)])
def test_factor_batch_matches_single_calls(m, n, s1, s2):
    print("factor_batch:", m, n, s1, s2, flush=True)
    k, seed = 5, 80
    V = torch.stack([torch.from_numpy(synth.make_V(m, n, 1e8, seed=seed + b)) for b in range(k)]).to("cuda")
    V[2, :, n // 2] = 0.0  # member 2 is rank deficient: its sketch has a zero pivot
    with rc.Plan(m, n, s1, s2, seed=seed, batch=k + 2) as pb:
        Q, R = pb.factor_batch(V)
        torch.cuda.synchronize()
        st = [pb.info_member(b) for b in range(k)]
        assert pb.info_batch(k) == st
        # a smaller batch on the same plan, in place (Q is V)
        Vi = V[:3].clone()
        Qi, Ri = pb.factor_batch(Vi, Q=Vi)
        torch.cuda.synchronize()
        st_i = [pb.info_member(b) for b in range(3)]
    # explicit, non-consecutive seeds (a device array)
    seeds = [900, 17, 4242, 5, 77][:k]
    with rc.Plan(m, n, s1, s2, seed=0, batch=k) as pb:
        Qx, Rx = pb.factor_batch(V, seeds=torch.tensor(seeds, dtype=torch.int64, device="cuda"))
        torch.cuda.synchronize()
        st_x = [pb.info_member(b) for b in range(k)]
    for b in (0, 3):
        with rc.Plan(m, n, s1, s2, seed=seeds[b]) as p:
            Qs, Rs = p.factor(V[b])
            torch.cuda.synchronize()
        assert st_x[b] == (rc.OK, 0)
        assert torch.equal(Qx[b], Qs) and torch.equal(Rx[b], Rs), ("seeds", b)
    for b in range(k):
        with rc.Plan(m, n, s1, s2, seed=seed + b) as p:
            Qs, Rs = p.factor(V[b], check=False)
            torch.cuda.synchronize()
            assert st[b] == p.info(), b
        if b == 2:
            assert st[b][0] == rc.E_RANK
            continue
        assert st[b] == (rc.OK, 0)
        assert torch.equal(Q[b], Qs) and torch.equal(R[b], Rs), b
        if b < 3:
            assert st_i[b] == st[b]
            assert torch.equal(Qi[b], Qs) and torch.equal(Ri[b], Rs), b
    torch.cuda.synchronize()


def test_factor_batch_limits():
    with rc.Plan(1000, 16, 512, 64, seed=1, batch=2) as p:
        V = torch.zeros((3, 1000, 16), dtype=torch.float64, device="cuda")
        with pytest.raises(rc.RcqrError):
            p.factor_batch(V)  # more members than the workspace holds
    with rc.Plan(1000, 100, 2000, 200, seed=1, batch=2, flags=rc.FLAG_REORTH) as p:
        V = torch.zeros((2, 1000, 100), dtype=torch.float64, device="cuda")
        with pytest.raises(rc.RcqrError) as e:
            p.factor_batch(V)  # plan flags: batches run the plain FP64 method only
        assert e.value.status == rc.E_UNSUPPORTED
    torch.cuda.synchronize()


def test_factor_batch_members_match_oracle():
    # members of one rcqr_factor_batch launch against the CPU oracle on their own seeds:
    # W1 (the workspace slice of member 0 is the plan's), R to 1e-10 (kappa <= 1e6), 10 n u bounds
    import numpy as np

    from oracle.rand_cholqr import U_PAPER, rand_cholqr as oracle_rand_cholqr

    for m, n, s1, s2 in [(10_000, 16, 512, 64), (20_001, 50, 5000, 200)]:
        k, seed = 4, 90
        print("factor_batch vs oracle:", m, n, s1, s2, flush=True)
        Vh = [synth.make_V(m, n, 10.0 ** (3 + b), seed=seed + b) for b in range(k)]
        V = torch.stack([torch.from_numpy(v) for v in Vh]).to("cuda")
        with rc.Plan(m, n, s1, s2, seed=seed, batch=k) as pb:
            Q, R = pb.factor_batch(V)
            torch.cuda.synchronize()
            assert pb.info_batch(k) == [(rc.OK, 0)] * k
            W1_0 = pb.intermediates()["W1"].cpu().numpy()
        tgt = 10 * n * U_PAPER
        for b in range(k):
            o = oracle_rand_cholqr(Vh[b], s1, s2, seed + b)
            assert o["status"] == 0
            if b == 0:
                assert np.linalg.norm(W1_0 - o["W1"]) <= 1e-13 * np.linalg.norm(o["W1"])
            Qb, Rb = Q[b].cpu().numpy(), R[b].cpu().numpy()
            assert np.linalg.norm(Rb - o["R"]) <= 1e-10 * np.linalg.norm(o["R"]), b
            assert np.linalg.norm(np.eye(n) - Qb.T @ Qb) <= tgt
            assert np.linalg.norm(Vh[b] - Qb @ Rb) / np.linalg.norm(Vh[b]) <= tgt
