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
