"""Continuous-batching request loop for rand_cholQR on one GPU.

Requests arrive over time; each is a matrix V already resident on the device plus its sketch
sizes and seed.  The loop admits a request as soon as it has arrived, a stream slot is free and
its HBM footprint (workspace + Q + R) fits in what the requests in flight leave of the budget,
in arrival order.  Admitted requests run on separate HIP streams, so their kernels overlap on the
device: one request's single-workgroup steps (Householder of the sketch, Cholesky) leave the
other compute units to the streaming passes of the others.  Completions are found by polling HIP
events; a request's latency is its device completion time minus its arrival time.

With max_batch > 1 the loop also batches when a backlog has built up (more requests waiting behind
the head than there are slots): when the head request is admitted, requests behind
it that have already arrived and have the same column shape (backend.shape_key: n, s1, s2) and a
row count within a factor of two of the head's (backend.joinable) join it, in arrival order, up to
max_batch and within the memory budget, and run as
one rcqr_factor_ragged launch on the slot (each with its own V, Q, R and seed; results bitwise
those of separate calls).  Requests of that shape can thereby start ahead of earlier requests of
other shapes; the head itself never waits.  Without a backlog, arrivals start on slots of their
own instead, which is faster for each of them (measured at 2000 arrivals/s: p50 0.8 ms against
1.6 ms when every chance to batch was taken).

The scheduling logic is independent of the GPU (`Scheduler` with a backend); `GpuBackend` runs
the factorizations through the C ABI, `serve()` wires the two together.
"""

import collections
import itertools
import time

import torch

from . import OK, Plan, workspace_bytes


class Scheduler:
    """FIFO admission by arrival time, free slot and memory budget.

    backend.footprint(req) -> bytes; backend.launch(req, slot) -> handle;
    backend.poll(handle) -> None while running, else (end_time_s, status).
    With max_batch > 1 also backend.shape_key(req) (None: never batched) and
    backend.launch_batch(reqs, slot) -> handle, whose poll gives (end_time_s, [status per request]).
    Times are seconds since the start of the run (backend.now() gives the current one).
    """

    def __init__(self, backend, slots, budget_bytes, max_batch=1):
        if slots < 1 or budget_bytes <= 0 or max_batch < 1:
            raise ValueError("need at least one slot, a positive memory budget and max_batch >= 1")
        self.backend, self.slots, self.budget = backend, int(slots), int(budget_bytes)
        self.max_batch = int(max_batch)

    def _followers(self, pending, head, now, room):
        """Arrived requests behind the head with its shape, in arrival order, that fit `room`."""
        if self.max_batch == 1:
            return []
        key = self.backend.shape_key(head)
        if key is None:
            return []
        out = []
        joinable = getattr(self.backend, "joinable", None)
        for idx in itertools.islice(pending, 1, None):
            if len(out) + 1 >= self.max_batch:
                break
            req = self.requests[idx]
            if req["arrival_s"] > now:
                break
            if self.backend.shape_key(req) == key and (joinable is None or joinable(head, req)):
                fp = self._footprint(idx)
                if fp <= room:
                    out.append(idx)
                    room -= fp
        return out

    def _footprint(self, idx):
        fp = self._fps.get(idx)
        if fp is None:
            fp = self._fps[idx] = self.backend.footprint(self.requests[idx])
        return fp

    def run(self, requests, idle_sleep_s=0.0):
        self.requests = requests
        self._fps = {}
        order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival_s"])
        pending = collections.deque(order)
        free_slots = list(range(self.slots))[::-1]
        inflight = {}
        used = 0
        peak_used, peak_inflight = 0, 0
        results = [None] * len(requests)
        while pending or inflight:
            progressed = False
            for key in list(inflight):
                slot, handle, fp, start, members = inflight[key]
                done = self.backend.poll(handle)
                if done is not None:
                    end, status = done
                    statuses = status if isinstance(status, list) else [status]
                    for idx, st in zip(members, statuses):
                        req = requests[idx]
                        results[idx] = {"index": idx, "arrival_s": req["arrival_s"], "start_s": start, "end_s": end,
                                        "latency_s": end - req["arrival_s"], "status": st, "slot": slot,
                                        "batch": len(members)}
                    del inflight[key]
                    free_slots.append(slot)
                    used -= fp
                    progressed = True
            now = self.backend.now()
            while pending and free_slots:
                idx = pending[0]
                req = requests[idx]
                if req["arrival_s"] > now:
                    break
                fp = self._footprint(idx)
                if fp > self.budget:
                    pending.popleft()
                    results[idx] = {"index": idx, "arrival_s": req["arrival_s"], "start_s": None, "end_s": None,
                                    "latency_s": None, "status": "rejected: footprint above the memory budget",
                                    "slot": None}
                    progressed = True
                    continue
                idle = self.backend.idle_bytes() if hasattr(self.backend, "idle_bytes") else 0
                if used + fp + idle > self.budget and idle > 0:
                    idle -= self.backend.evict_idle(used + fp + idle - self.budget)
                if used + fp + idle > self.budget:
                    break  # wait for memory; keep arrival order
                pending.popleft()
                slot = free_slots.pop()
                group = []
                if self.max_batch > 1:
                    # batch only under a backlog: more requests waiting behind the head than there are
                    # slots (below that, each starts on a slot of its own soon, which is faster for it)
                    waiting = 0
                    for i in pending:
                        if requests[i]["arrival_s"] > now or waiting > self.slots:
                            break
                        waiting += 1
                    if waiting > self.slots:
                        group = self._followers(collections.deque([idx]) + pending, req, now, self.budget - used - fp - idle)
                if group:
                    for g in group:
                        pending.remove(g)
                    members = [idx] + group
                    fp += sum(self._footprint(g) for g in group)
                    handle = self.backend.launch_batch([requests[i] for i in members], slot)
                else:
                    members = [idx]
                    handle = self.backend.launch(req, slot)
                inflight[idx] = (slot, handle, fp, now, members)
                used += fp
                peak_used = max(peak_used, used)
                peak_inflight = max(peak_inflight, sum(len(v[4]) for v in inflight.values()))
                progressed = True
            if not progressed and idle_sleep_s > 0:
                time.sleep(idle_sleep_s)
        return {"results": results, "peak_bytes": peak_used, "peak_inflight": peak_inflight}


class GpuBackend:
    """Runs requests through the C ABI on one HIP stream per slot; V comes from get_V(req), either a
    tensor whose contents are complete when get_V returns, or (tensor, event) with a HIP event
    (torch.cuda.Event) recorded after the work that writes it, which the slot's stream waits for.
    (Waiting on the caller's whole stream instead would record an event on the legacy default
    stream, which orders it after the work of every slot: measured, it serialised the slots and
    tripled the p50 latency.)

    Requests of one column shape (n, s1, s2; plain FP64) admitted together share
    rcqr_factor_ragged launches whatever their row counts: each member reads its own V and writes
    its own Q and R (no copy of V), and is bitwise the result of a single rcqr_factor with its
    seed.  A request admitted alone runs rcqr_factor on a plan of its own shape (measured at 2000
    arrivals/s: p50 0.8 ms this way against 1.5 ms through a one-member ragged launch).  Plans are cached per
    (slot, column shape), at most plans_per_slot per slot, least recently used evicted; a cached
    plan holds batch_hint workspace slices sized for m_cap rows (or more when a request needs
    it) and is remade larger when a batch needs more.  With plan flags (single-precision sketch,
    second Cholesky QR) every request gets a plan of its own.  A slot runs one launch at a time
    and is handed back only after its launch has completed, so its cached plans and seed buffers
    are free whenever the scheduler launches on it.

    Memory: footprint(req) counts what a request holds while in flight (its Q and R and its
    workspace slice at the cached plans' row count); idle_bytes() counts the workspace slices
    cached plans keep beyond the launches in flight, and evict_idle(nbytes) frees least recently
    used idle plans; the scheduler admits a request only while in-flight footprints plus idle
    plans fit the budget, evicting idle plans when that makes the room."""

    def __init__(self, get_V, slots, device="cuda:0", flags=0, keep_outputs=False, batch_hint=1, plans_per_slot=4, m_cap=0,
                 batching=True):
        self.device = torch.device(device)
        self.batching = bool(batching)
        self.batch_plans = {}
        self.batch_hint = max(1, int(batch_hint))
        self.plans_per_slot = max(1, int(plans_per_slot))
        self.m_cap = int(m_cap)
        self.get_V = get_V
        self.flags = flags
        self.keep = keep_outputs  # True: every request's (Q, R) by seed; a set of seeds: those requests' only
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.busy = set()  # slots with a launch in flight
        self.outputs = {}
        self.reset_clock()

    def reset_clock(self):
        """Start the run's clock now (after everything queued so far has finished)."""
        torch.cuda.synchronize(self.device)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.streams[0])
        self.t0_event.synchronize()
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def _plan_rows(self, req):
        return max(self.m_cap, req["m"])

    def footprint(self, req):
        m, n = req["m"], req["n"]
        mw = self._plan_rows(req) if self.shape_key(req) is not None else m
        return workspace_bytes(mw, n, req["s1"], req["s2"], self.flags) + 8 * m * n + 8 * n * n

    def idle_bytes(self):
        """Workspace bytes of cached plans beyond what the launches in flight use."""
        return sum(p.workspace.numel() for (slot, _), p in self.batch_plans.items() if slot not in self.busy)

    def evict_idle(self, nbytes):
        """Free least recently used cached plans of idle slots until nbytes are freed (or none left)."""
        freed = 0
        for key in list(self.batch_plans):
            if freed >= nbytes:
                break
            if key[0] in self.busy:
                continue
            p = self.batch_plans.pop(key)
            freed += p.workspace.numel()
            p.close()
        return freed

    def close(self):
        for p in self.batch_plans.values():
            p.close()
        self.batch_plans = {}

    def shape_key(self, req):
        """Requests with equal keys can share one rcqr_factor_ragged launch (plain FP64, any m);
        None (a plan and an rcqr_factor call per request) with flags or with batching off."""
        if self.flags != 0 or not self.batching:
            return None
        return (req["n"], req["s1"], req["s2"])

    def joinable(self, head, req):
        """A follower joins the head's launch only with a row count within a factor of two of the
        head's: a batch ends with its largest member, so a small request batched behind a large
        one would wait for it."""
        return req["m"] <= 2 * head["m"] and head["m"] <= 2 * req["m"]

    def _batch_plan(self, slot, key, count, m_need):
        """The slot's cached plan for `key`, made (or remade larger) when it cannot hold `count`
        members of up to m_need rows."""
        cached = self.batch_plans.pop((slot, key), None)
        if cached is None or cached.batch < count or cached.m < m_need:
            m_plan = max(m_need, self.m_cap, cached.m if cached is not None else 0)
            count = max(count, cached.batch if cached is not None else 0)
            if cached is not None:
                cached.close()
            mine = [k for k in self.batch_plans if k[0] == slot]
            while len(mine) >= self.plans_per_slot:  # dict order = least recently used first
                self.batch_plans.pop(mine.pop(0)).close()
            n, s1, s2 = key
            cached = Plan(m_plan, n, s1, s2, 0, device=self.device, stream=self.streams[slot], batch=max(count, self.batch_hint))
        self.batch_plans[(slot, key)] = cached  # (re)inserted last: most recently used
        return cached

    def _inputs(self, reqs, stream):
        """The requests' V; the slot stream waits for the ones that come with a readiness event."""
        Vs = []
        for r in reqs:
            got = self.get_V(r)
            if isinstance(got, tuple):
                V, ready = got
                if ready is not None:
                    stream.wait_event(ready)
            else:
                V = got
            Vs.append(V)
        return Vs

    def launch(self, req, slot):
        # a request without followers takes a plan of its own shape (the ragged launch pays for
        # its member table and for the batch plan's capacity)
        stream = self.streams[slot]
        V = self._inputs([req], stream)[0]
        self.busy.add(slot)
        with torch.cuda.stream(stream):
            plan = Plan(req["m"], req["n"], req["s1"], req["s2"], req["seed"], device=self.device, stream=stream,
                        flags=self.flags)
            Q = torch.empty((req["m"], req["n"]), dtype=torch.float64, device=self.device)
            R = torch.empty((req["n"], req["n"]), dtype=torch.float64, device=self.device)
            plan.factor(V, Q, R, check=False)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        return {"req": req, "plan": plan, "Q": Q, "R": R, "V": V, "event": done, "slot": slot}

    def launch_batch(self, reqs, slot):
        stream = self.streams[slot]
        key = self.shape_key(reqs[0])
        Vs = self._inputs(reqs, stream)
        self.busy.add(slot)
        with torch.cuda.stream(stream):
            plan = self._batch_plan(slot, key, len(reqs), max(r["m"] for r in reqs))
            Qs, Rs = plan.factor_ragged(Vs, seeds=[r["seed"] for r in reqs])
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        return {"reqs": reqs, "plan": plan, "Q": Qs, "R": Rs, "V": Vs, "event": done, "slot": slot}

    def _kept(self, seed):
        return self.keep is True or (not isinstance(self.keep, bool) and seed in self.keep)

    def poll(self, handle):
        if not handle["event"].query():
            return None
        end = self.t0_event.elapsed_time(handle["event"]) * 1e-3
        self.busy.discard(handle["slot"])
        if "reqs" in handle:  # a batch (its plan stays cached for the slot)
            sts = [st for st, _ in handle["plan"].info_batch(len(handle["reqs"]))]
            for b, r in enumerate(handle["reqs"]):
                if self._kept(r["seed"]):
                    self.outputs[r["seed"]] = (handle["Q"][b], handle["R"][b])
            return end, sts
        st, _ = handle["plan"].info()
        if self._kept(handle["req"]["seed"]):
            self.outputs[handle["req"]["seed"]] = (handle["Q"], handle["R"])
        handle["plan"].close()
        return end, st


def latency_summary(run):
    """p50 / p99 latency (s) and completed requests per second over the run."""
    done = [r for r in run["results"] if r is not None and r["end_s"] is not None]
    lat = sorted(r["latency_s"] for r in done)
    if not lat:
        return {"completed": 0}

    def pct(p):
        k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[k]

    span = max(r["end_s"] for r in done) - min(r["arrival_s"] for r in done)
    ok = sum(1 for r in done if r["status"] == OK)
    return {"completed": len(done), "ok": ok, "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
            "mean_ms": 1e3 * sum(lat) / len(lat), "qr_per_s": len(done) / span if span > 0 else None,
            "peak_bytes": run["peak_bytes"], "peak_inflight": run["peak_inflight"]}


def serve(requests, get_V, slots=4, budget_bytes=32 << 30, device="cuda:0", flags=0, keep_outputs=False, max_batch=1,
          backend=None, m_cap=0, batching=True):
    """Run the request list with continuous batching; returns (run, summary, backend).

    With `backend` (a GpuBackend with at least `slots` streams) the run reuses it and its cached
    plans, restarting its clock; the caller closes it.  Otherwise a new one is made and closed."""
    own = backend is None
    if own:
        backend = GpuBackend(get_V, slots, device=device, flags=flags, keep_outputs=keep_outputs, batch_hint=max_batch, m_cap=m_cap,
                             batching=batching)
    else:
        if slots > len(backend.streams):
            raise ValueError(f"{slots} slots need as many streams; the backend has {len(backend.streams)}")
        backend.get_V = get_V
        backend.reset_clock()
    run = Scheduler(backend, slots, budget_bytes, max_batch=max_batch).run(requests)
    torch.cuda.synchronize(backend.device)
    if own:
        backend.close()
    return run, latency_summary(run), backend
