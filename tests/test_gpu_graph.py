"""HIP-graph replays of a factorization (rcqr_graph_*) against eager calls of the same plan:
every replay gives bitwise the eager Q and R, with eager work on the same plan and stream in
between (the workspace is shared), for rand_cholQR, cholQR2 and sCholQR3, 16 to 128 columns."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


@pytest.mark.parametrize("m,n,s1,s2,method,kappa", [(10_000, 16, 512, 64, "rand_cholqr", 1e4),
                                                    (30_000, 64, 8192, 256, "rand_cholqr", 1e12),
                                                    (20_000, 100, 20_000, 400, "rand_cholqr", 1e10),
                                                    (20_000, 32, 2048, 128, "cholqr2", 1e4),
                                                    (20_000, 64, 8192, 256, "scholqr3", 1e8)])
def test_graph_replays_match_eager(m, n, s1, s2, method, kappa):
    print("graph:", m, n, method, flush=True)
    stream = torch.cuda.Stream()
    V = torch.from_numpy(synth.make_V(m, n, kappa, seed=n)).to("cuda")
    V2 = torch.from_numpy(synth.make_V(m, n, 1e3, seed=n + 1)).to("cuda")
    with torch.cuda.stream(stream):
        p = rc.Plan(m, n, s1, s2, seed=7, stream=stream)
        eager = getattr(p, {"rand_cholqr": "factor"}.get(method, method))
        Qe, Re = eager(V)
        Qe, Re = Qe.clone(), Re.clone()
        g = p.graph(V, method=method)
        for rep in range(3):
            g.Q.fill_(float("nan"))
            g.R.fill_(float("nan"))
            g.launch()
            stream.synchronize()
            assert p.info() == (rc.OK, 0)
            assert torch.equal(g.Q, Qe) and torch.equal(g.R, Re), rep
            # eager work on the same plan (same workspace) between replays
            Q2, R2 = eager(V2)
            stream.synchronize()
            assert not torch.equal(R2, Re)
        g.close()
        p.close()
    torch.cuda.synchronize()
