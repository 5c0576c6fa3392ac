"""Host logic of the continuous-batching loop (no GPU): a simulated backend with known service
times checks admission order, the slot and memory limits, and the latency bookkeeping."""

import pytest

from paper_2309_05868_amd.serve import Scheduler, latency_summary


class FakeBackend:
    """Simulated clock: it advances by one tick on every poll and every read of the time, so the
    loop never waits on the wall clock."""

    def __init__(self, tick=1e-4):
        self.t = 0.0
        self.tick = tick
        self.launched = []
        self.inflight_bytes = 0
        self.max_bytes = 0

    def now(self):
        self.t += self.tick
        return self.t

    def footprint(self, req):
        return req["bytes"]

    def launch(self, req, slot):
        self.launched.append((req["id"], slot, self.t))
        self.inflight_bytes += req["bytes"]
        self.max_bytes = max(self.max_bytes, self.inflight_bytes)
        return {"req": req, "end": self.t + req["work"]}

    def poll(self, h):
        self.t += self.tick
        if self.t >= h["end"]:
            if not h.get("done"):
                h["done"] = True
                self.inflight_bytes -= h["req"]["bytes"]
            return h["end"], 0
        return None


def reqs(spec):
    return [{"id": i, "arrival_s": a, "work": w, "bytes": b} for i, (a, w, b) in enumerate(spec)]


def test_fifo_admission_within_slots_and_budget():
    spec = [(0.000, 0.010, 40), (0.001, 0.010, 40), (0.002, 0.010, 40), (0.003, 0.001, 10), (0.050, 0.002, 90)]
    be = FakeBackend()
    run = Scheduler(be, slots=3, budget_bytes=100).run(reqs(spec))
    order = [i for i, _, _ in be.launched]
    assert order == [0, 1, 2, 3, 4]          # arrival order, never overtaken
    assert be.max_bytes <= 100               # memory budget held
    starts = {i: t for i, _, t in be.launched}
    assert starts[2] >= 0.010 - 1e-9         # third 40-byte request waited for memory
    assert starts[3] >= starts[2]            # FIFO: the small one behind it waited too
    res = run["results"]
    assert all(r["status"] == 0 for r in res)
    for r in res:
        assert r["end_s"] >= r["start_s"] >= r["arrival_s"]
        assert r["latency_s"] == pytest.approx(r["end_s"] - r["arrival_s"])
    assert run["peak_inflight"] <= 3


def test_slots_limit_concurrency_and_oversized_requests_are_rejected():
    spec = [(0.0, 0.005, 1)] * 6 + [(0.0, 0.001, 1000)]
    be = FakeBackend()
    run = Scheduler(be, slots=2, budget_bytes=100).run(reqs(spec))
    assert run["peak_inflight"] == 2
    res = run["results"]
    assert res[6]["status"].startswith("rejected")
    s = latency_summary(run)
    assert s["completed"] == 6 and s["ok"] == 6
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_more_slots_lower_latency():
    spec = [(0.0005 * i, 0.004, 1) for i in range(40)]
    one = latency_summary(Scheduler(FakeBackend(), slots=1, budget_bytes=10**9).run(reqs(spec)))
    four = latency_summary(Scheduler(FakeBackend(), slots=4, budget_bytes=10**9).run(reqs(spec)))
    assert four["p99_ms"] < one["p99_ms"]
    assert four["qr_per_s"] > one["qr_per_s"]


def test_invalid_configuration():
    with pytest.raises(ValueError):
        Scheduler(FakeBackend(), slots=0, budget_bytes=10)


class FakeBatchBackend(FakeBackend):
    """Adds batched launches: a batch takes the longest member's work; shape = req["shape"]."""

    def __init__(self, tick=1e-4):
        super().__init__(tick)
        self.batches = []

    def shape_key(self, req):
        return req.get("shape")

    def launch_batch(self, reqs, slot):
        self.batches.append([r["id"] for r in reqs])
        self.launched.extend((r["id"], slot, self.t) for r in reqs)
        b = sum(r["bytes"] for r in reqs)
        self.inflight_bytes += b
        self.max_bytes = max(self.max_bytes, self.inflight_bytes)
        return {"req": {"bytes": b}, "end": self.t + max(r["work"] for r in reqs), "n": len(reqs)}

    def poll(self, h):
        done = super().poll(h)
        if done is None or "n" not in h:
            return done
        return done[0], [0] * h["n"]


def test_same_shape_requests_share_a_launch():
    # ids 0..5 arrive together; shapes A A B A B A; one slot busy-free; max_batch 3
    spec = [(0.0, 0.002, 10)] * 6
    rq = reqs(spec)
    for r, sh in zip(rq, "AABABA"):
        r["shape"] = sh
    be = FakeBatchBackend()
    run = Scheduler(be, slots=1, budget_bytes=10**6, max_batch=3).run(rq)
    # the head (0) takes the next two arrived A's (1, 3); then 2 takes 4; then 5 alone
    assert be.batches == [[0, 1, 3], [2, 4], [5]] or be.batches[:2] == [[0, 1, 3], [2, 4]]
    res = run["results"]
    assert all(r["status"] == 0 for r in res)
    assert res[0]["batch"] == 3 and res[2]["batch"] == 2


def test_no_batching_without_a_backlog():
    # two same-shape arrivals and two slots: each starts on its own slot; with four arrivals and
    # two slots (three waiting behind the head) the head takes the others along
    spec = [(0.0, 0.002, 10)] * 2
    rq = reqs(spec)
    for r in rq:
        r["shape"] = "A"
    be = FakeBatchBackend()
    run = Scheduler(be, slots=2, budget_bytes=10**6, max_batch=4).run(rq)
    assert be.batches == []  # both went through single launches
    assert sorted(slot for _, slot, _ in be.launched) == [0, 1]
    assert all(r["batch"] == 1 for r in run["results"])
    rq = reqs([(0.0, 0.002, 10)] * 4)
    for r in rq:
        r["shape"] = "A"
    be = FakeBatchBackend()
    Scheduler(be, slots=2, budget_bytes=10**6, max_batch=4).run(rq)
    assert be.batches[0] == [0, 1, 2, 3]


def test_batches_respect_budget_and_unbatchable_requests():
    spec = [(0.0, 0.002, 40)] * 4
    rq = reqs(spec)
    for r in rq:
        r["shape"] = "A"
    rq[1]["shape"] = None  # never batched
    be = FakeBatchBackend()
    Scheduler(be, slots=2, budget_bytes=100, max_batch=4).run(rq)
    assert be.max_bytes <= 100
    for b in be.batches:
        assert 1 not in b or len(b) == 1
    assert all(len(b) <= 2 for b in be.batches)  # 40-byte members: at most two fit 100 bytes


class _FakePlan:
    made = []

    def __init__(self, m, n, s1, s2, seed, device=None, stream=None, batch=1):
        self.m, self.key, self.batch, self.closed = m, (n, s1, s2), batch, False
        self.workspace = _FakeWorkspace(1000 * m * batch)
        _FakePlan.made.append(self)

    def close(self):
        self.closed = True


class _FakeWorkspace:
    def __init__(self, nbytes):
        self.nbytes = nbytes

    def numel(self):
        return self.nbytes


def _fake_backend(srv, batch_hint=2, plans_per_slot=2, m_cap=0):
    be = object.__new__(srv.GpuBackend)
    be.batch_plans, be.batch_hint, be.plans_per_slot, be.m_cap = {}, batch_hint, plans_per_slot, m_cap
    be.device, be.streams, be.busy, be.flags, be.batching = None, [None, None], set(), 0, True
    return be


def test_gpu_backend_plan_cache_is_lru_per_slot(monkeypatch):
    # host logic of the per-slot plan cache (keyed by column shape), with a stand-in Plan
    from paper_2309_05868_amd import serve as srv

    monkeypatch.setattr(srv, "Plan", _FakePlan)
    _FakePlan.made = []
    be = _fake_backend(srv)
    A, B, C = (8, 128, 32), (16, 512, 64), (32, 2048, 128)
    assert be.shape_key({"n": 8, "s1": 128, "s2": 32, "m": 5}) == A   # any row count
    pa = be._batch_plan(0, A, 1, 100)
    assert pa.batch == 2 and pa.m == 100                 # sized for the batch hint and the rows
    assert be._batch_plan(0, A, 2, 80) is pa             # reused while it holds count and rows
    pb = be._batch_plan(0, B, 1, 100)
    pb1 = be._batch_plan(1, B, 1, 100)                   # other slot: its own plan
    assert pb1 is not pb
    assert be._batch_plan(0, A, 1, 100) is pa            # A used last on slot 0, so B is the oldest
    pc = be._batch_plan(0, C, 1, 100)                    # third shape on slot 0 evicts B only
    assert pb.closed and not pa.closed and not pc.closed and not pb1.closed
    assert set(be.batch_plans) == {(0, A), (0, C), (1, B)}
    pa4 = be._batch_plan(0, A, 4, 100)                   # too few members: remade larger
    assert pa.closed and pa4.batch == 4 and not pc.closed
    pa5 = be._batch_plan(0, A, 1, 300)                   # too few rows: remade with more
    assert pa4.closed and pa5.m == 300 and pa5.batch == 4
    be.close()
    assert all(p.closed for p in _FakePlan.made) and be.batch_plans == {}


def test_gpu_backend_idle_plans_counted_and_evicted(monkeypatch):
    from paper_2309_05868_amd import serve as srv

    monkeypatch.setattr(srv, "Plan", _FakePlan)
    be = _fake_backend(srv, batch_hint=1, m_cap=10)
    A, B = (8, 128, 32), (16, 512, 64)
    pa = be._batch_plan(0, A, 1, 10)
    pb = be._batch_plan(1, B, 1, 10)
    assert be.idle_bytes() == pa.workspace.numel() + pb.workspace.numel()
    be.busy.add(1)                                        # slot 1 has a launch in flight
    assert be.idle_bytes() == pa.workspace.numel()
    assert be.evict_idle(1) == pa.workspace.numel()       # only the idle slot's plan goes
    assert pa.closed and not pb.closed and be.idle_bytes() == 0


def test_serve_rejects_more_slots_than_backend_streams():
    from paper_2309_05868_amd import serve as srv

    be = object.__new__(srv.GpuBackend)
    be.streams = [None, None]
    with pytest.raises(ValueError):
        srv.serve([], lambda r: None, slots=3, backend=be)


def test_gpu_backend_keeps_outputs_of_selected_seeds():
    # host logic of output retention: every request's outputs, none, or those of a set of seeds
    from paper_2309_05868_amd import serve as srv

    be = _fake_backend(srv)
    for keep, kept in ((True, {1, 2, 3}), (False, set()), ({2, 9}, {2})):
        be.keep = keep
        assert {s for s in (1, 2, 3) if be._kept(s)} == kept
