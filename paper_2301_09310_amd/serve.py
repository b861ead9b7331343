"""Serving loop: continuous batching of alignment requests on one GPU.

Requests (batches of pairs of any size) arrive over time and wait in FIFO
order.  Whenever an execution slot is free, the loop forms one launch from
the head of the queue: every waiting request that still fits the launch's
pair and byte capacity and the HBM budget next to the work already on the
GPU.  A launch is one call of the library's default (persistent,
length-binned) path over the merged pairs of its requests, on the slot's
own HIP stream.  So at low load a request starts alone as soon as it
arrives, and under load the requests that arrived while earlier launches
ran are aligned together: their pairs share one work queue and one
length-binned schedule, and the new launch overlaps the tail of the
running ones on the device.

Merging needs no repacking: each request's packed streams are copied
byte-aligned into the slot's pinned staging buffers, its offsets are
shifted by the byte position, and one pad pair after each request (its
query and target are the few padding bases up to the next request's
first sequences) keeps the merged offsets contiguous; its output is
dropped.  Staging and device buffers (the slot's device arena: sequences,
offsets and the pair-to-request tags) are allocated once per slot, so the
steady state allocates nothing.

Completion is per request: the launch goes through salo_align_batch_tagged,
whose kernel writes each pair's answers straight into the slot's host
result buffer (host memory the device writes coherently) and then adds 1
to its request's counter there.  The loop polls the counters and hands a
request its results as soon as its own pairs are done, while the rest of
the merged launch still runs; the slot itself is reused when the whole
launch has ended (one HIP event).  Latency is measured from each request's
scheduled arrival (open loop, so a slow server cannot hide queueing
delay).

The control plane (admission, FIFO order, launch forming, accounting) only
talks to an executor object, so it runs on the CPU with a fake executor
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
    status: str = "pending"            # pending | running | done | rejected
    result: tuple | None = None        # (score, q_end, t_end) numpy int32
    footprint: int = 0
    launch: int = -1                   # index of the launch that ran it

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival if self.t_done >= 0 else float("nan")


def footprint_bytes(batch) -> int:
    """Device bytes one request holds while in flight: packed sequences,
    offsets (one more entry for the pad pair), outputs, and the plan's
    per-pair buffers (keys and order)."""
    n = batch.n_pairs + 1
    return int(batch.q_seqs.nbytes + batch.t_seqs.nbytes + 16 * (n + 1) + 12 * n + 6 * n)


class Merged:
    """Byte-aligned concatenation of several requests' packed pairs, with
    one pad pair after each request (see the module docstring)."""

    def __init__(self, batches):
        self.batches = list(batches)
        self.q_bytes = sum(b.q_seqs.nbytes for b in self.batches)
        self.t_bytes = sum(b.t_seqs.nbytes for b in self.batches)
        self.n_pairs = sum(b.n_pairs + 1 for b in self.batches)

    def fill(self, q, qo, t, to):
        """Write the merged streams into q/t (uint8) and the offsets into
        qo/to (int64, n_pairs + 1 entries); returns each request's first
        output index.  The pad pair after a request spans the padding bases
        between its last sequences and the next request's first ones (a few
        bases of each stream; its result is not used)."""
        starts = []
        bq = bt = p = 0
        for b in self.batches:
            n = b.n_pairs
            q[bq:bq + b.q_seqs.nbytes] = b.q_seqs
            t[bt:bt + b.t_seqs.nbytes] = b.t_seqs
            qo[p:p + n + 1] = b.q_offsets + 4 * bq
            to[p:p + n + 1] = b.t_offsets + 4 * bt
            starts.append(p)
            bq += b.q_seqs.nbytes
            bt += b.t_seqs.nbytes
            p += n + 1
            qo[p] = 4 * bq
            to[p] = 4 * bt
        return starts


# Each request's completion counter gets its own 128-byte line (tags step
# by 32 counters): the device's system-scope increments of one line are
# serialised, and with adjacent counters a merged launch ran 20% longer.
TAG_STRIDE = 32


class GpuExecutor:
    """Runs launches on `n_slots` HIP streams, each with buffers sized for
    `max_pairs` pairs and `max_bytes` packed bytes per sequence stream.
    per_request: signal each request's completion as its own pairs finish
    (salo_align_batch_tagged); otherwise the launch's end completes all of
    its requests."""

    def __init__(self, n_slots: int = 3, max_pairs: int = 1 << 17,
                 max_bytes: int = 96 << 20, scoring=(1, -4, 6, 1), device="cuda",
                 per_request: bool = True, split_waves: int = 0,
                 split_max_long: int = 1024, **options):
        import torch
        from paper_2301_09310_amd import salo
        salo.load()
        self.torch, self.salo = torch, salo
        self.device = torch.device(device)
        self.scoring = scoring
        self.options = options
        self.per_request = per_request
        # long pairs (queries above 1024 bases) run on split_waves waves each
        # when a launch holds at most split_max_long of them: then the GPU
        # has room for every split unit at once and the split only shortens
        # the launch; with more, splitting would cost throughput
        self.split_waves = int(split_waves)
        self.split_max_long = int(split_max_long)
        self.launch_split = []
        self.max_pairs = int(max_pairs)
        self.max_bytes = int(max_bytes)
        self.slots = []
        for _ in range(n_slots):
            s = torch.cuda.Stream(device=self.device)
            host = {"q": torch.empty(self.max_bytes, dtype=torch.uint8, pin_memory=True),
                    "t": torch.empty(self.max_bytes, dtype=torch.uint8, pin_memory=True),
                    "qo": torch.empty(self.max_pairs + 1, dtype=torch.int64, pin_memory=True),
                    "to": torch.empty(self.max_pairs + 1, dtype=torch.int64, pin_memory=True)}
            if per_request:
                host["tag"] = torch.empty(self.max_pairs, dtype=torch.int32, pin_memory=True)
            else:
                host["out"] = torch.empty((3, self.max_pairs), dtype=torch.int32,
                                          pin_memory=True)
            dev = {k: torch.empty_like(v, device=self.device) for k, v in host.items()}
            slot = {"stream": s, "host": host, "dev": dev, "event": torch.cuda.Event()}
            if per_request:
                # results and per-request counters in coherent host memory:
                # the kernel writes them, the loop reads them while it runs
                slot["res"] = salo.HostBuffer(3 * self.max_pairs, np.int32)
                # a request takes at least one pair and one pad pair
                slot["done"] = salo.HostBuffer((self.max_pairs // 2 + 1) * TAG_STRIDE,
                                               np.uint32)
            salo.reserve(self.max_pairs, stream=s)
            self.slots.append(slot)
        self.free = list(range(n_slots))

    @property
    def slots_free(self) -> int:
        return len(self.free)

    def fits(self, n_pairs: int, q_bytes: int, t_bytes: int) -> bool:
        """Whether a launch of this size fits one slot."""
        return n_pairs <= self.max_pairs and q_bytes <= self.max_bytes \
            and t_bytes <= self.max_bytes

    def submit(self, reqs):
        torch = self.torch
        k = self.free.pop()
        sl = self.slots[k]
        m = Merged([r.batch for r in reqs])
        h, d, s = sl["host"], sl["dev"], sl["stream"]
        n = m.n_pairs
        starts = m.fill(h["q"].numpy(), h["qo"].numpy(), h["t"].numpy(), h["to"].numpy())
        if self.per_request:
            tag = h["tag"].numpy()
            for i, (r, p) in enumerate(zip(reqs, starts)):
                tag[p:p + r.batch.n_pairs] = i * TAG_STRIDE
                tag[p + r.batch.n_pairs] = -1          # the pad pair after the request
            sl["done"].array[:len(reqs) * TAG_STRIDE] = 0
        # the stream waits for the previous launch on this slot before the
        # staging copies overwrite its device buffers (stream order)
        opts = dict(self.options)
        if self.split_waves > 1:
            n_long = sum(int((r.batch.q_lens() > 1024).sum()) for r in reqs)
            if n_long <= self.split_max_long:
                opts["split_waves"] = self.split_waves
            self.launch_split.append(opts.get("split_waves", 0))
        with torch.cuda.stream(s):
            d["q"][:m.q_bytes].copy_(h["q"][:m.q_bytes], non_blocking=True)
            d["t"][:m.t_bytes].copy_(h["t"][:m.t_bytes], non_blocking=True)
            d["qo"][:n + 1].copy_(h["qo"][:n + 1], non_blocking=True)
            d["to"][:n + 1].copy_(h["to"][:n + 1], non_blocking=True)
            if self.per_request:
                d["tag"][:n].copy_(h["tag"][:n], non_blocking=True)
                base = sl["res"].ptr
                outs = (base, base + 4 * self.max_pairs, base + 8 * self.max_pairs)
                self.salo.align_batch_tagged(d["q"][:m.q_bytes], d["qo"][:n + 1],
                                             d["t"][:m.t_bytes], d["to"][:n + 1], self.scoring,
                                             outs, d["tag"], sl["done"].ptr, stream=s, **opts)
            else:
                out = (d["out"][0, :n], d["out"][1, :n], d["out"][2, :n])
                self.salo.align_batch(d["q"][:m.q_bytes], d["qo"][:n + 1], d["t"][:m.t_bytes],
                                      d["to"][:n + 1], self.scoring, out=out, stream=s, **opts)
                for c in range(3):
                    h["out"][c, :n].copy_(d["out"][c, :n], non_blocking=True)
            sl["event"].record(s)
        return (k, [(r, p) for r, p in zip(reqs, starts)], set())

    def _result(self, sl, r, p):
        if self.per_request:
            res = sl["res"].array
            n = r.batch.n_pairs
            mp = self.max_pairs
            return tuple(res[c * mp + p:c * mp + p + n].copy() for c in range(3))
        out = sl["host"]["out"].numpy()
        return tuple(out[c, p:p + r.batch.n_pairs].copy() for c in range(3))

    def poll_requests(self, handle):
        """Requests of a running launch whose pairs have all finished since
        the last poll: [(index in the launch, result)]."""
        if not self.per_request:
            return []
        k, parts, reported = handle
        sl = self.slots[k]
        done = sl["done"].array
        out = []
        for i, (r, p) in enumerate(parts):
            if i not in reported and int(done[i * TAG_STRIDE]) == r.batch.n_pairs:
                reported.add(i)
                out.append((i, self._result(sl, r, p)))
        return out

    def poll(self, handle) -> bool:
        return self.slots[handle[0]]["event"].query()

    def collect(self, handle):
        """Wait for the launch's end, free its slot and return every
        request's result."""
        k, parts, _ = handle
        sl = self.slots[k]
        sl["event"].synchronize()
        res = [self._result(sl, r, p) for r, p in parts]
        self.free.append(k)
        return res


@dataclass
class ServeStats:
    completed: int = 0
    rejected: int = 0
    cells: int = 0
    first_arrival: float = 0.0
    last_done: float = 0.0
    max_inflight_bytes: int = 0
    max_inflight: int = 0              # requests on the GPU at once
    max_launches: int = 0              # launches on the GPU at once
    launches: int = 0
    launch_sizes: list = field(default_factory=list)   # requests per launch
    latencies: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([float("nan")])
        span = max(self.last_done - self.first_arrival, 1e-12)
        sizes = np.array(self.launch_sizes) if self.launch_sizes else np.zeros(1)
        return {"completed": self.completed, "rejected": self.rejected,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(np.mean(lat) * 1e3),
                "gcups": self.cells / span / 1e9,
                "requests_per_s": self.completed / span,
                "launches": self.launches,
                "mean_requests_per_launch": float(sizes.mean()),
                "max_inflight_bytes": self.max_inflight_bytes,
                "max_inflight": self.max_inflight,
                "max_launches": self.max_launches}


class Server:
    """FIFO admission by HBM footprint into merged launches that overlap on
    the device (continuous batching)."""

    def __init__(self, executor, budget_bytes: int, clock=time.perf_counter,
                 sleep=time.sleep, poll_interval: float = 50e-6, progress=None,
                 progress_every: float = 5.0):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.clock = clock
        self.sleep = sleep
        self.poll_interval = poll_interval
        self.progress = progress
        self.progress_every = progress_every

    def _form_launch(self, pending, in_bytes):
        """Take requests from the head of the queue while the launch fits
        one slot and the budget; returns (launch, rejected)."""
        take, rejected = [], []
        nb = q_b = t_b = fp = 0
        while pending:
            head = pending[0]
            b = head.batch
            alone_fits = self.ex.fits(b.n_pairs + 1, b.q_seqs.nbytes, b.t_seqs.nbytes) \
                and head.footprint <= self.budget
            if not alone_fits:
                rejected.append(pending.pop(0))
                continue
            if not self.ex.fits(nb + b.n_pairs + 1, q_b + b.q_seqs.nbytes,
                                t_b + b.t_seqs.nbytes) \
                    or in_bytes + fp + head.footprint > self.budget:
                break
            take.append(pending.pop(0))
            nb += b.n_pairs + 1
            q_b += b.q_seqs.nbytes
            t_b += b.t_seqs.nbytes
            fp += head.footprint
        return take, rejected

    def run(self, requests, warmup: int = 0) -> ServeStats:
        """Serve `requests` (arrival times relative to the start).  The
        first `warmup` requests by arrival are served but left out of the
        stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival += t0
            r.footprint = footprint_bytes(r.batch)
        stats = ServeStats()
        pending, inflight = [], []          # inflight: (handle, [requests])
        nxt = in_bytes = done_count = 0
        last_report = t0
        while done_count < len(reqs):
            now = self.clock()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            # completions: requests whose own pairs are done (executors that
            # signal per request), then whole launches
            still = []
            per_req = getattr(self.ex, "poll_requests", None)
            for handle, group in inflight:
                if per_req is not None:
                    for i, res in per_req(handle):
                        r = group[i]
                        r.result, r.t_done, r.status = res, self.clock(), "done"
                        done_count += 1
                if self.ex.poll(handle):
                    results = self.ex.collect(handle)
                    t_done = self.clock()
                    for r, res in zip(group, results):
                        if r.status != "done":
                            r.result, r.t_done, r.status = res, t_done, "done"
                            done_count += 1
                        in_bytes -= r.footprint
                else:
                    still.append((handle, group))
            inflight = still
            # form launches while slots are free
            while pending and self.ex.slots_free > 0:
                take, rejected = self._form_launch(pending, in_bytes)
                for r in rejected:
                    r.status, r.t_done = "rejected", self.clock()
                    done_count += 1
                if not take:
                    break
                t_admit = self.clock()
                for r in take:
                    r.t_admit, r.status, r.launch = t_admit, "running", stats.launches
                    in_bytes += r.footprint
                inflight.append((self.ex.submit(take), take))
                stats.launches += 1
                stats.launch_sizes.append(len(take))
                stats.max_inflight_bytes = max(stats.max_inflight_bytes, in_bytes)
                stats.max_inflight = max(stats.max_inflight, sum(len(g) for _, g in inflight))
                stats.max_launches = max(stats.max_launches, len(inflight))
            if self.progress is not None and self.clock() - last_report >= self.progress_every:
                last_report = self.clock()
                self.progress("served %d/%d requests, %d launches, %d waiting"
                              % (done_count, len(reqs), stats.launches, len(pending)))
            if done_count < len(reqs):
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


def with_arrivals(requests, arrivals):
    """Fresh requests sharing the batches of `requests`, with new arrival
    times (the same requests replayed at another offered rate)."""
    return [Request(rid=r.rid, batch=r.batch, arrival=float(t))
            for r, t in zip(requests, arrivals)]


def split_requests(pool, sizes, arrivals):
    """Requests carved from consecutive pairs of a pool batch."""
    out, p = [], 0
    for k, (sz, t) in enumerate(zip(sizes, arrivals)):
        idx = np.arange(p, p + sz) % pool.n_pairs
        p += sz
        out.append(Request(rid=k, batch=pool.subset(idx), arrival=float(t)))
    return out
