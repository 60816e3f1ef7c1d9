"""Serving loop for k-input multiplies: continuous batching under an HBM budget.

Requests (ring degree, k, level, input ciphertexts already on the device)
arrive over time.  The server keeps the evaluation keys of every parameter
set resident, admits waiting requests in arrival order while their device
memory (multiply workspace + output) fits what the HBM budget leaves after
the resident state, and launches the admitted requests as one micro-batch
on a free stream while earlier micro-batches are still running.  A
micro-batch holds one job-table plan per ring degree (every stage one launch
over all of that degree's requests, see mick_jobs_plan), smallest degree
first, each followed by its own completion event, so light requests do not
wait for a heavy one of a larger degree.  When a plan's event has fired its
requests' memory returns to the budget and their latency (completion minus
arrival) is recorded; the stream is free again when its last plan is done.

The scheduler is host code and talks to the device through an executor, so
its policy can be tested on the CPU with FakeExecutor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    rid: int
    log_n: int
    k: int
    level: int
    arrival: float          # seconds after the start of the run
    inputs: object = None   # executor-specific handle of the k input ciphertexts
    nbytes: int = 0         # device memory while in flight (set by the server)
    start: Optional[float] = None
    done: Optional[float] = None
    output: object = None


class Executor:
    """What the server needs from the device side."""

    n_streams = 2

    def request_bytes(self, req: Request) -> int:
        """Device memory one request holds from admission to completion."""
        raise NotImplementedError

    def launch(self, reqs: List[Request], slot: int) -> List[tuple]:
        """Start a micro-batch on stream `slot`; returns [(token, requests)],
        one entry per independently completing group."""
        raise NotImplementedError

    def poll(self, token) -> Optional[float]:
        """Completion time (seconds after start) once the group is done, else None."""
        raise NotImplementedError

    def now(self) -> float:
        raise NotImplementedError

    def wait_until(self, t: float) -> None:
        raise NotImplementedError


@dataclasses.dataclass
class ServeStats:
    completed: List[Request]
    peak_bytes: int
    micro_batches: int
    wall: float

    def latencies(self):
        return [r.done - r.arrival for r in self.completed]

    def summary(self) -> Dict[str, float]:
        import numpy as np
        lat = np.array(self.latencies()) * 1e3
        span = max(r.done for r in self.completed) - min(r.arrival for r in self.completed)
        return {"requests": len(self.completed), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
                "max_ms": round(float(lat.max()), 3), "ct_mults_per_s": round(len(self.completed) / span, 2),
                "micro_batches": self.micro_batches, "peak_inflight_gb": round(self.peak_bytes / 1e9, 3)}


class Server:
    """Continuous-batching scheduler.

    budget: bytes of device memory the server may hold in all; resident:
    bytes already held for the whole run (keys, input state), so in-flight
    requests get budget - resident.  max_batch: most requests per
    micro-batch."""

    def __init__(self, executor: Executor, budget: int, resident: int = 0, max_batch: int = 256):
        if resident >= budget:
            raise ValueError("resident state alone exceeds the HBM budget")
        self.ex = executor
        self.budget = budget - resident
        self.max_batch = max_batch

    def run(self, requests: Sequence[Request]) -> ServeStats:
        for r in requests:
            r.nbytes = self.ex.request_bytes(r)
            if r.nbytes > self.budget:
                raise ValueError("request %d needs more memory than the budget leaves" % r.rid)
        arrivals = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque = collections.deque()
        groups = []                      # [token, slot, requests]
        open_groups = collections.Counter()  # slot -> groups still running
        free_slots = list(range(self.ex.n_streams))
        used = peak = batches = 0
        done: List[Request] = []
        t_wall = time.perf_counter()
        while arrivals or waiting or groups:
            now = self.ex.now()
            while arrivals and arrivals[0].arrival <= now:
                waiting.append(arrivals.popleft())
            still = []
            for g in groups:
                t = self.ex.poll(g[0])
                if t is None:
                    still.append(g)
                    continue
                for r in g[2]:
                    r.done = t
                    used -= r.nbytes
                    done.append(r)
                open_groups[g[1]] -= 1
                if open_groups[g[1]] == 0:
                    free_slots.append(g[1])
            groups = still
            if waiting and free_slots:
                batch = []
                while waiting and len(batch) < self.max_batch and used + waiting[0].nbytes <= self.budget:
                    r = waiting.popleft()
                    used += r.nbytes
                    r.start = now
                    batch.append(r)
                if batch:
                    peak = max(peak, used)
                    slot = free_slots.pop(0)
                    for tok, reqs in self.ex.launch(batch, slot):
                        groups.append([tok, slot, reqs])
                        open_groups[slot] += 1
                    batches += 1
                    continue
            if not waiting and not groups and arrivals:
                self.ex.wait_until(arrivals[0].arrival)
        return ServeStats(done, peak, batches, time.perf_counter() - t_wall)


def poisson_arrivals(n: int, rate: float, seed: int) -> List[float]:
    """Open-loop arrival times of n requests at `rate` per second."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [float(t) for t in np.cumsum(rng.exponential(1.0 / rate, n))]


class GpuExecutor(Executor):
    """Runs micro-batches through job-table plans on `n_streams` streams.

    params / keys: dicts log_n -> mick.Params / mick.Keys, resident for the
    whole run.  Request.inputs is the list of k input tensors [2, level, N].
    Outputs are released with their plan unless `keep(request)` is true."""

    def __init__(self, mick, torch, params, keys, n_streams: int = 2, keep=None):
        self.mick, self.torch = mick, torch
        self.params, self.keys = params, keys
        self.n_streams = n_streams
        self.keep = keep  # predicate: keep this request's output tensor in Request.output
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.t0_event = None
        self.t0 = None
        self.host_launch_s = 0.0

    def start(self):
        """Zero of both clocks: a GPU event and the host time right after it."""
        torch = self.torch
        torch.cuda.synchronize()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        self.host_launch_s = 0.0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        while self.now() < t:
            time.sleep(min(5e-5, max(0.0, t - self.now())))

    def request_bytes(self, req: Request) -> int:
        prm = self.params[req.log_n]
        out = 2 * (req.level - req.k + 1) * prm.N * 4
        ws = self.mick.jobs_workspace_bytes(prm, [(req.k, req.level)])
        return ws + out

    def launch(self, reqs: List[Request], slot: int):
        torch, mick = self.torch, self.mick
        stream = self.streams[slot]
        by_n: Dict[int, List[Request]] = collections.defaultdict(list)
        for r in reqs:
            by_n[r.log_n].append(r)
        out = []
        t = time.perf_counter()
        with torch.cuda.stream(stream):
            # every job table is written before the first kernel of this
            # micro-batch is queued, so no table copy waits behind kernels
            plans = [(mick.Plan(self.params[ln], self.keys[ln], [(r.inputs, r.level, None) for r in by_n[ln]]),
                      by_n[ln]) for ln in sorted(by_n)]
            for plan, rs in plans:
                plan.run()
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(stream)
                if self.keep is not None:
                    for r, o in zip(rs, plan.outs):
                        if self.keep(r):
                            r.output = o
                # the plan (and with it the workspace and outputs) lives until the event has fired
                out.append(((ev, plan), rs))
        self.host_launch_s += time.perf_counter() - t
        return out

    def poll(self, token) -> Optional[float]:
        ev, _plan = token
        if not ev.query():
            return None
        return self.t0_event.elapsed_time(ev) / 1e3


class FakeExecutor(Executor):
    """Host-only stand-in with a deterministic clock: a group finishes
    cost(requests) seconds after both its launch and the previous group on
    the same stream; streams run in parallel.  Each host step costs `tick`."""

    def __init__(self, n_streams: int = 2, bytes_fn=None, cost_fn=None, tick: float = 1e-5):
        self.n_streams = n_streams
        self.t = 0.0
        self.tick = tick
        self.bytes_fn = bytes_fn or (lambda r: 1000 * r.k * r.level)
        self.cost_fn = cost_fn or (lambda rs: 1e-3 * sum(r.k for r in rs))
        self.stream_end = [0.0] * n_streams
        self.launched = []   # (slot, start, end, [rid])

    def now(self) -> float:
        self.t += self.tick
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def request_bytes(self, req: Request) -> int:
        return self.bytes_fn(req)

    def launch(self, reqs, slot):
        by_n = collections.defaultdict(list)
        for r in reqs:
            by_n[r.log_n].append(r)
        out = []
        for ln in sorted(by_n):
            start = max(self.t, self.stream_end[slot])
            end = start + self.cost_fn(by_n[ln])
            self.stream_end[slot] = end
            self.launched.append((slot, start, end, [r.rid for r in by_n[ln]]))
            out.append((end, by_n[ln]))
        return out

    def poll(self, token):
        return token if self.t >= token else None


def request_mix(n: int, seed: int, sets: Dict[int, tuple], heavy_frac: float = 0.1):
    """(log_n, k, level) of n requests: with probability heavy_frac a heavy
    request (largest ring degree, k = min(12, L), level uniform in [k, L]); otherwise
    N uniform over `sets` (log_n -> (L, K, dnum)), k uniform in
    [2, min(12, L)], level uniform in [k, L]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    top = max(sets)
    out = []
    for _ in range(n):
        if rng.random() < heavy_frac:
            L = sets[top][0]
            k = min(12, L)
            out.append((top, k, int(rng.integers(k, L + 1))))
            continue
        ln = int(rng.choice(sorted(sets)))
        L = sets[ln][0]
        k = int(rng.integers(2, min(12, L) + 1))
        out.append((ln, k, int(rng.integers(k, L + 1))))
    return out
