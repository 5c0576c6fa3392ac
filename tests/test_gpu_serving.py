"""Continuous batching on the GPU: requests of uneven m, n and kappa served concurrently on
several streams give bitwise the same Q and R as each request factored alone (the kernels do
not depend on what else runs), and every result meets the 10 n u bounds."""

import numpy as np
import pytest
import torch

import synth
from oracle.rand_cholqr import U_PAPER, rand_cholqr as oracle_rand_cholqr

pytestmark = pytest.mark.gpu

rc = pytest.importorskip("paper_2309_05868_amd")
from paper_2309_05868_amd import serve as srv  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc.lib()


def check_against_oracle(reqs, outputs, Vs, count):
    """Served Q and R of up to `count` requests with kappa <= 1e6 (smallest first) against the CPU
    oracle on the request's seed: R to 1e-10 relative, Q to 1e-10 * max(1, kappa / 1e4)."""
    sample = sorted((r for r in reqs if r["kappa"] <= 1e6), key=lambda r: r["m"] * r["n"])[:count]
    assert sample, "no request with kappa <= 1e6 to compare"
    for r in sample:
        Qs, Rs = outputs[r["seed"]]
        Qh, Rh = Qs.cpu().numpy(), Rs.cpu().numpy()
        o = oracle_rand_cholqr(Vs[r["seed"]].cpu().numpy(), r["s1"], r["s2"], r["seed"])
        assert o["status"] == 0
        assert np.linalg.norm(Rh - o["R"]) <= 1e-10 * np.linalg.norm(o["R"]), r
        assert np.linalg.norm(Qh - o["Q"]) <= 1e-10 * max(1.0, r["kappa"] / 1e4) * np.linalg.norm(o["Q"]), r


def test_served_results_equal_solo_results():
    reqs = synth.make_requests(24, seed=77, rate_per_s=20_000.0, m_range=(2000, 40_000),
                               n_choices=(8, 16, 32, 64, 100, 128), kappa_range=(1e2, 1e12))
    Vs = {}
    for r in reqs:
        Vs[r["seed"]] = torch.from_numpy(synth.make_V(r["m"], r["n"], r["kappa"], r["seed"])).to("cuda")
    print("serving: 24 requests on 4 streams", flush=True)
    run, summary, backend = srv.serve(reqs, lambda r: Vs[r["seed"]], slots=4, budget_bytes=4 << 30, keep_outputs=True)
    print("serving summary", summary, flush=True)
    assert summary["completed"] == 24 and summary["ok"] == 24
    assert summary["peak_inflight"] > 1  # requests did overlap
    for r in reqs:
        Qs, Rs = backend.outputs[r["seed"]]
        with rc.Plan(r["m"], r["n"], r["s1"], r["s2"], r["seed"]) as p:
            Q, R = p.factor(Vs[r["seed"]])
        torch.cuda.synchronize()
        assert torch.equal(Q, Qs) and torch.equal(R, Rs), r
        n = r["n"]
        Qh, Rh, Vh = Q.cpu().numpy(), R.cpu().numpy(), Vs[r["seed"]].cpu().numpy()
        tgt = 10 * n * U_PAPER
        assert np.linalg.norm(np.eye(n) - Qh.T @ Qh) <= tgt
        assert np.linalg.norm(Vh - Qh @ Rh) / np.linalg.norm(Vh) <= tgt
    check_against_oracle(reqs, backend.outputs, Vs, 5)


def test_memory_budget_serialises_requests():
    reqs = synth.make_requests(6, seed=78, rate_per_s=1e6, m_range=(5000, 6000), n_choices=(64,),
                               kappa_range=(1e3, 1e3))
    Vs = {r["seed"]: torch.from_numpy(synth.make_V(r["m"], r["n"], r["kappa"], r["seed"])).to("cuda") for r in reqs}
    one = max(rc.workspace_bytes(r["m"], r["n"], r["s1"], r["s2"]) + 8 * r["m"] * r["n"] + 8 * r["n"] ** 2 for r in reqs)
    run, summary, _ = srv.serve(reqs, lambda r: Vs[r["seed"]], slots=4, budget_bytes=one)
    assert summary["completed"] == 6 and summary["ok"] == 6
    assert run["peak_inflight"] == 1 and run["peak_bytes"] <= one


def test_same_shape_requests_batched_equal_solo_results():
    # 40 requests of three shapes arriving together: the loop groups same-shaped ones into
    # rcqr_factor_batch launches (per-request seeds); each result is bitwise the solo result
    shapes = [(10_000, 16, 512, 64), (5000, 8, 128, 32), (20_000, 64, 8192, 256)]
    reqs = []
    for i in range(40):
        m, n, s1, s2 = shapes[i % 3]
        reqs.append({"arrival_s": 0.0, "m": m, "n": n, "s1": s1, "s2": s2, "seed": 500 + 7 * i, "kappa": 1e6})
    Vs = {r["seed"]: torch.from_numpy(synth.make_V(r["m"], r["n"], r["kappa"], r["seed"])).to("cuda") for r in reqs}
    print("serving: 40 requests, batches of up to 8", flush=True)
    run, summary, backend = srv.serve(reqs, lambda r: Vs[r["seed"]], slots=2, budget_bytes=8 << 30, keep_outputs=True,
                                      max_batch=8)
    print("serving summary", summary, flush=True)
    assert summary["completed"] == 40 and summary["ok"] == 40
    assert max(r["batch"] for r in run["results"]) > 1  # some requests shared a launch
    for r in reqs:
        Qs, Rs = backend.outputs[r["seed"]]
        with rc.Plan(r["m"], r["n"], r["s1"], r["s2"], r["seed"]) as p:
            Q, R = p.factor(Vs[r["seed"]])
        torch.cuda.synchronize()
        assert torch.equal(Q, Qs) and torch.equal(R, Rs), r
    check_against_oracle([r for r in reqs if r["n"] <= 16], backend.outputs, Vs, 4)


def test_reused_backend_with_plan_evictions_equals_solo_results():
    # two runs on one backend whose slots cache one plan each: shapes alternate, so cached plans
    # are evicted and remade between launches; every result is bitwise the solo result
    shapes = [(6000, 16, 512, 64), (4000, 32, 2048, 128), (3000, 8, 128, 32)]
    runs = []
    for rep in range(2):
        reqs = []
        for i in range(12):
            m, n, s1, s2 = shapes[(i + rep) % 3]
            reqs.append({"arrival_s": 1e-4 * i, "m": m, "n": n, "s1": s1, "s2": s2, "seed": 900 + 31 * i + rep,
                         "kappa": 1e8})
        runs.append(reqs)
    Vs = {r["seed"]: torch.from_numpy(synth.make_V(r["m"], r["n"], r["kappa"], r["seed"])).to("cuda")
          for reqs in runs for r in reqs}
    be = srv.GpuBackend(lambda r: Vs[r["seed"]], 2, keep_outputs=True, batch_hint=4, plans_per_slot=1)
    try:
        for reqs in runs:
            print("serving: 12 requests on a reused backend", flush=True)
            run, summary, _ = srv.serve(reqs, lambda r: Vs[r["seed"]], slots=2, budget_bytes=4 << 30, max_batch=4,
                                        backend=be)
            assert summary["completed"] == 12 and summary["ok"] == 12
            assert len(be.batch_plans) <= 2
    finally:
        be.close()
    for reqs in runs:
        for r in reqs:
            Qs, Rs = be.outputs[r["seed"]]
            with rc.Plan(r["m"], r["n"], r["s1"], r["s2"], r["seed"]) as p:
                Q, R = p.factor(Vs[r["seed"]])
            torch.cuda.synchronize()
            assert torch.equal(Q, Qs) and torch.equal(R, Rs), r


def test_request_with_readiness_event_waits_for_its_producer():
    # V is written on another stream behind a spin; get_V hands over (V, event) and the served
    # result must be that of the finished V (the slot stream waits for the event)
    reqs = [{"arrival_s": 0.0, "m": 20_000 + 1000 * i, "n": 16, "s1": 512, "s2": 64, "seed": 700 + i, "kappa": 1e6}
            for i in range(3)]
    src = {r["seed"]: torch.from_numpy(synth.make_V(r["m"], r["n"], r["kappa"], r["seed"])).to("cuda") for r in reqs}
    dst = {k: torch.zeros_like(v) for k, v in src.items()}
    torch.cuda.synchronize()
    prod = torch.cuda.Stream()
    ready = {}
    with torch.cuda.stream(prod):
        for k in dst:
            torch.cuda._sleep(20_000_000)  # a bounded spin: the copy lands well after the launch
            dst[k].copy_(src[k])
            ev = torch.cuda.Event()
            ev.record(prod)
            ready[k] = ev
    run, summary, backend = srv.serve(reqs, lambda r: (dst[r["seed"]], ready[r["seed"]]), slots=2, budget_bytes=4 << 30,
                                      keep_outputs=True, max_batch=4)
    assert summary["completed"] == 3 and summary["ok"] == 3
    for r in reqs:
        Qs, Rs = backend.outputs[r["seed"]]
        with rc.Plan(r["m"], r["n"], r["s1"], r["s2"], r["seed"]) as p:
            Q, R = p.factor(src[r["seed"]])
        torch.cuda.synchronize()
        assert torch.equal(Q, Qs) and torch.equal(R, Rs), r
