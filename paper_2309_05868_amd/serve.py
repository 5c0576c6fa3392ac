"""Continuous-batching request loop for rand_cholQR on one GPU.

Requests arrive over time; each is a matrix V already resident on the device plus its sketch
sizes and seed.  The loop admits a request as soon as it has arrived, a stream slot is free and
its HBM footprint (workspace + Q + R) fits in what the requests in flight leave of the budget,
in arrival order.  Admitted requests run on separate HIP streams, so their kernels overlap on the
device: one request's single-workgroup steps (Householder of the sketch, Cholesky) leave the
other compute units to the streaming passes of the others.  Completions are found by polling HIP
events; a request's latency is its device completion time minus its arrival time.

The scheduling logic is independent of the GPU (`Scheduler` with a backend); `GpuBackend` runs
the factorizations through the C ABI, `serve()` wires the two together.
"""

import collections
import time

import torch

from . import OK, Plan, workspace_bytes


class Scheduler:
    """FIFO admission by arrival time, free slot and memory budget.

    backend.footprint(req) -> bytes; backend.launch(req, slot) -> handle;
    backend.poll(handle) -> None while running, else (end_time_s, status).
    Times are seconds since the start of the run (backend.now() gives the current one).
    """

    def __init__(self, backend, slots, budget_bytes):
        if slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive memory budget")
        self.backend, self.slots, self.budget = backend, int(slots), int(budget_bytes)

    def run(self, requests, idle_sleep_s=0.0):
        order = sorted(range(len(requests)), key=lambda i: requests[i]["arrival_s"])
        pending = collections.deque(order)
        free_slots = list(range(self.slots))[::-1]
        inflight = {}
        used = 0
        peak_used, peak_inflight = 0, 0
        results = [None] * len(requests)
        while pending or inflight:
            progressed = False
            for idx in list(inflight):
                slot, handle, fp, start = inflight[idx]
                done = self.backend.poll(handle)
                if done is not None:
                    end, status = done
                    req = requests[idx]
                    results[idx] = {"index": idx, "arrival_s": req["arrival_s"], "start_s": start, "end_s": end,
                                    "latency_s": end - req["arrival_s"], "status": status, "slot": slot}
                    del inflight[idx]
                    free_slots.append(slot)
                    used -= fp
                    progressed = True
            now = self.backend.now()
            while pending and free_slots:
                idx = pending[0]
                req = requests[idx]
                if req["arrival_s"] > now:
                    break
                fp = self.backend.footprint(req)
                if fp > self.budget:
                    pending.popleft()
                    results[idx] = {"index": idx, "arrival_s": req["arrival_s"], "start_s": None, "end_s": None,
                                    "latency_s": None, "status": "rejected: footprint above the memory budget",
                                    "slot": None}
                    progressed = True
                    continue
                if used + fp > self.budget:
                    break  # wait for memory; keep arrival order
                pending.popleft()
                slot = free_slots.pop()
                handle = self.backend.launch(req, slot)
                inflight[idx] = (slot, handle, fp, now)
                used += fp
                peak_used = max(peak_used, used)
                peak_inflight = max(peak_inflight, len(inflight))
                progressed = True
            if not progressed and idle_sleep_s > 0:
                time.sleep(idle_sleep_s)
        return {"results": results, "peak_bytes": peak_used, "peak_inflight": peak_inflight}


class GpuBackend:
    """Runs each request as one rcqr_factor on a slot's stream; V comes from get_V(req)."""

    def __init__(self, get_V, slots, device="cuda:0", flags=0, keep_outputs=False):
        self.device = torch.device(device)
        self.get_V = get_V
        self.flags = flags
        self.keep = keep_outputs
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.outputs = {}
        torch.cuda.synchronize(self.device)
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.streams[0])
        self.t0_event.synchronize()
        self.t0_host = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0_host

    def footprint(self, req):
        m, n = req["m"], req["n"]
        return workspace_bytes(m, n, req["s1"], req["s2"], self.flags) + 8 * m * n + 8 * n * n

    def launch(self, req, slot):
        stream = self.streams[slot]
        V = self.get_V(req)
        with torch.cuda.stream(stream):
            plan = Plan(req["m"], req["n"], req["s1"], req["s2"], req["seed"], device=self.device, stream=stream,
                        flags=self.flags)
            Q = torch.empty((req["m"], req["n"]), dtype=torch.float64, device=self.device)
            R = torch.empty((req["n"], req["n"]), dtype=torch.float64, device=self.device)
            plan.factor(V, Q, R, check=False)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        return {"req": req, "plan": plan, "Q": Q, "R": R, "event": done}

    def poll(self, handle):
        if not handle["event"].query():
            return None
        end = self.t0_event.elapsed_time(handle["event"]) * 1e-3
        st, _ = handle["plan"].info()
        if self.keep:
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


def serve(requests, get_V, slots=4, budget_bytes=32 << 30, device="cuda:0", flags=0, keep_outputs=False):
    """Run the request list with continuous batching; returns (run, summary, backend)."""
    backend = GpuBackend(get_V, slots, device=device, flags=flags, keep_outputs=keep_outputs)
    run = Scheduler(backend, slots, budget_bytes).run(requests)
    torch.cuda.synchronize(backend.device)
    return run, latency_summary(run), backend
