"""Serving control plane on the CPU: admission by footprint, FIFO order,
overlap, rejection and latency accounting, with a fake executor (answers
from the oracle, takes time proportional to cells on a fake clock)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I
from paper_2301_09310_amd import serve as S


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """n_slots concurrent slots; a request finishes `cells / rate` seconds
    after submission; results come from the oracle."""

    def __init__(self, clock, n_slots=2, rate=1e6):
        self.clock, self.rate = clock, rate
        self.free = n_slots
        self.order = []

    @property
    def slots_free(self):
        return self.free

    def submit(self, req):
        self.free -= 1
        self.order.append(req.rid)
        return (self.clock() + req.batch.cells() / self.rate, req)

    def poll(self, handle):
        return self.clock() >= handle[0]

    def collect(self, handle):
        self.free += 1
        b = handle[1].batch
        return O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)


def _requests(n, max_pairs=20, rate=50.0, seed=3):
    pool = I.random_pairs(seed, 400, 60)
    sizes = S.request_sizes(n, seed, max_pairs)
    arr = S.poisson_arrivals(n, rate, seed)
    return S.split_requests(pool, sizes, arr)


def test_fifo_with_one_slot():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=1)
    reqs = _requests(30)
    st = S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs)
    assert ex.order == sorted(ex.order)           # admitted in arrival order
    assert st.completed == 30 and st.max_inflight == 1
    done = [r.t_done for r in sorted(reqs, key=lambda r: r.rid)]
    assert done == sorted(done)                   # and completed in order


def test_budget_is_never_exceeded_and_work_overlaps():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=8, rate=2e5)
    reqs = _requests(60, rate=400.0)
    budget = 3 * max(S.footprint_bytes(r.batch) for r in reqs)
    st = S.Server(ex, budget_bytes=budget, clock=clk, sleep=clk.sleep).run(reqs)
    assert st.max_inflight_bytes <= budget
    assert st.max_inflight >= 2                   # requests ran concurrently
    assert st.completed == 60


def test_request_larger_than_budget_is_rejected():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=2)
    reqs = _requests(10)
    big = max(reqs, key=lambda r: S.footprint_bytes(r.batch))
    budget = S.footprint_bytes(big.batch) - 1
    st = S.Server(ex, budget_bytes=budget, clock=clk, sleep=clk.sleep).run(reqs)
    assert big.status == "rejected"
    assert st.completed + st.rejected == 10


def test_latency_counts_from_scheduled_arrival():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=1, rate=1e5)
    reqs = _requests(20, rate=1e4)                 # arrivals far faster than service
    st = S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs)
    for r in reqs:
        service = r.batch.cells() / 1e5
        assert r.latency >= service - 1e-6
    lat = np.array(st.latencies)
    assert lat[-1] > lat[0]                       # queueing delay builds up
    s = st.summary()
    assert s["p99_ms"] >= s["p50_ms"]


def test_results_are_the_oracle_answers():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=3)
    reqs = _requests(15)
    S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs)
    for r in reqs:
        b = r.batch
        want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
        for g, w in zip(r.result, want):
            assert np.array_equal(g, w)


def test_warmup_requests_are_excluded():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=2)
    reqs = _requests(25)
    st = S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs, warmup=5)
    assert st.completed == 20 and len(st.latencies) == 20
