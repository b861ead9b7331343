"""Serving loop: continuous batching of alignment requests on one GPU.

Requests (batches of pairs of any size) arrive over time.  The loop keeps
arrived requests in FIFO order and admits the head whenever its HBM
footprint fits the budget next to the requests already on the GPU and an
execution slot (a HIP stream) is free.  Each admitted request is copied to
the device and aligned on its own stream with the library's default
(persistent, length-binned) path, so requests that arrive while others run
start as soon as slots and memory free up and overlap on the device.
Results come back to pinned host memory; completion is observed through a
HIP event per request.  Latency is measured from the request's scheduled
arrival (open loop, so a slow server cannot hide queueing delay).

The control plane (admission, FIFO order, accounting) only talks to an
executor object, so it can be exercised on the CPU with a fake executor
and a fake clock.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    batch: object                      # inputs.Batch (packed host arrays)
    arrival: float                     # scheduled arrival time (seconds)
    t_admit: float = -1.0
    t_done: float = -1.0
    status: str = "pending"            # pending | running | done | rejected | failed
    result: tuple | None = None        # (score, q_end, t_end) numpy int32
    handle: object = None
    footprint: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival if self.t_done >= 0 else float("nan")


def footprint_bytes(batch) -> int:
    """Device bytes one request holds while in flight: packed sequences,
    offsets, outputs, and the plan's per-pair buffers (keys and order)."""
    n = batch.n_pairs
    return int(batch.q_seqs.nbytes + batch.t_seqs.nbytes + 16 * (n + 1) + 12 * n + 6 * n)


class GpuExecutor:
    """Runs each request on its own HIP stream through the library."""

    def __init__(self, n_streams: int = 4, scoring=(1, -4, 6, 1), device="cuda", **options):
        import torch
        from paper_2301_09310_amd import salo
        salo.load()
        self.torch, self.salo = torch, salo
        self.device = torch.device(device)
        self.scoring = scoring
        self.options = options
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.free = list(range(n_streams))

    @property
    def slots_free(self) -> int:
        return len(self.free)

    def reserve(self, max_pairs: int):
        for s in self.streams:
            self.salo.reserve(max_pairs, stream=s)

    def submit(self, req: Request):
        torch = self.torch
        k = self.free.pop()
        s = self.streams[k]
        b = req.batch
        n = b.n_pairs
        host_in = [torch.from_numpy(a).pin_memory() for a in
                   (b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)]
        host_out = [torch.empty(n, dtype=torch.int32).pin_memory() for _ in range(3)]
        with torch.cuda.stream(s):
            dev_in = [x.to(self.device, non_blocking=True) for x in host_in]
            dev_out = [torch.empty(n, dtype=torch.int32, device=self.device) for _ in range(3)]
            self.salo.align_batch(*dev_in, self.scoring, out=dev_out, stream=s, **self.options)
            for h, d in zip(host_out, dev_out):
                h.copy_(d, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # keep every buffer alive until the event has passed
        return (k, ev, host_in, dev_in, dev_out, host_out)

    def poll(self, handle) -> bool:
        return handle[1].query()

    def collect(self, handle):
        k, ev, _, _, _, host_out = handle
        ev.synchronize()
        self.free.append(k)
        return tuple(h.numpy().copy() for h in host_out)


@dataclass
class ServeStats:
    completed: int = 0
    rejected: int = 0
    cells: int = 0
    first_arrival: float = 0.0
    last_done: float = 0.0
    max_inflight_bytes: int = 0
    max_inflight: int = 0
    latencies: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([float("nan")])
        span = max(self.last_done - self.first_arrival, 1e-12)
        return {"completed": self.completed, "rejected": self.rejected,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(np.mean(lat) * 1e3),
                "gcups": self.cells / span / 1e9,
                "requests_per_s": self.completed / span,
                "max_inflight_bytes": self.max_inflight_bytes,
                "max_inflight": self.max_inflight}


class Server:
    """Admission by HBM footprint, FIFO order, overlapping execution."""

    def __init__(self, executor, budget_bytes: int, clock=time.perf_counter,
                 sleep=time.sleep, poll_interval: float = 50e-6):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.clock = clock
        self.sleep = sleep
        self.poll_interval = poll_interval

    def run(self, requests, warmup: int = 0) -> ServeStats:
        """Serve `requests` (sorted by arrival, times relative to the start).
        The first `warmup` requests are served but left out of the stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival += t0
            r.footprint = footprint_bytes(r.batch)
        stats = ServeStats()
        pending, inflight = [], []
        nxt, in_bytes = 0, 0
        done_count = 0
        while done_count < len(reqs):
            now = self.clock()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            # completions
            still = []
            for r in inflight:
                if self.ex.poll(r.handle):
                    r.result = self.ex.collect(r.handle)
                    r.t_done = self.clock()
                    r.status = "done"
                    r.handle = None
                    in_bytes -= r.footprint
                    done_count += 1
                else:
                    still.append(r)
            inflight = still
            # FIFO admission while the head fits
            while pending:
                head = pending[0]
                if head.footprint > self.budget:
                    head.status = "rejected"
                    head.t_done = self.clock()
                    pending.pop(0)
                    done_count += 1
                    continue
                if self.ex.slots_free == 0 or in_bytes + head.footprint > self.budget:
                    break
                pending.pop(0)
                head.t_admit = self.clock()
                head.status = "running"
                head.handle = self.ex.submit(head)
                in_bytes += head.footprint
                inflight.append(head)
                stats.max_inflight_bytes = max(stats.max_inflight_bytes, in_bytes)
                stats.max_inflight = max(stats.max_inflight, len(inflight))
            if done_count < len(reqs):
                # nothing changed this turn: wait a little (next arrival or
                # a completion)
                wait = self.poll_interval
                if not inflight and not pending and nxt < len(reqs):
                    wait = max(0.0, reqs[nxt].arrival - self.clock())
                self.sleep(wait)
        measured = reqs[warmup:]
        stats.first_arrival = min(r.arrival for r in measured) if measured else t0
        for r in measured:
            if r.status == "done":
                stats.completed += 1
                stats.cells += r.batch.cells()
                stats.latencies.append(r.latency)
                stats.last_done = max(stats.last_done, r.t_done)
            elif r.status == "rejected":
                stats.rejected += 1
        return stats


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng([seed, 9])
    return np.cumsum(rng.exponential(1.0 / rate, n))


def request_sizes(n: int, seed: int, max_pairs: int = 4096) -> np.ndarray:
    rng = np.random.default_rng([seed, 10])
    return rng.integers(1, max_pairs + 1, n)


def split_requests(pool, sizes, arrivals):
    """Requests carved from consecutive pairs of a pool batch."""
    out, p = [], 0
    for k, (sz, t) in enumerate(zip(sizes, arrivals)):
        idx = np.arange(p, p + sz) % pool.n_pairs
        p += sz
        out.append(Request(rid=k, batch=pool.subset(idx), arrival=float(t)))
    return out
