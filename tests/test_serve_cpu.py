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
    """n_slots concurrent launch slots; a launch finishes `cells / rate`
    seconds after submission; results come from the oracle."""

    def __init__(self, clock, n_slots=2, rate=1e6, max_pairs=1 << 20):
        self.clock, self.rate = clock, rate
        self.free = n_slots
        self.max_pairs = max_pairs
        self.order = []
        self.launches = []

    @property
    def slots_free(self):
        return self.free

    def fits(self, n_pairs, q_bytes, t_bytes):
        return n_pairs <= self.max_pairs

    def submit(self, reqs):
        self.free -= 1
        self.order += [r.rid for r in reqs]
        self.launches.append([r.rid for r in reqs])
        cells = sum(r.batch.cells() for r in reqs)
        return (self.clock() + cells / self.rate, reqs)

    def poll(self, handle):
        return self.clock() >= handle[0]

    def collect(self, handle):
        self.free += 1
        return [O.align_batch(r.batch.q_seqs, r.batch.q_offsets, r.batch.t_seqs,
                              r.batch.t_offsets) for r in handle[1]]


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
    assert st.completed == 30 and st.max_launches == 1
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


def test_waiting_requests_merge_into_one_launch():
    """With one slot busy, the requests that arrive meanwhile are aligned
    together in the next launch, in arrival order."""
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=1, rate=1e5)
    reqs = _requests(40, rate=2e3)
    st = S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs)
    assert st.completed == 40
    assert max(len(g) for g in ex.launches) > 1
    assert st.launches < 40
    assert [rid for g in ex.launches for rid in g] == list(range(40))
    for r in reqs:                                 # a launch completes all its requests
        mates = [x for x in reqs if x.launch == r.launch]
        assert all(x.t_done == r.t_done for x in mates)


def test_launch_capacity_splits_the_queue():
    clk = FakeClock()
    ex = FakeExecutor(clk, n_slots=2, rate=1e5, max_pairs=45)
    reqs = _requests(30, max_pairs=20, rate=1e5)
    st = S.Server(ex, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep).run(reqs)
    assert st.completed == 30
    by_id = {r.rid: r for r in reqs}
    for g in ex.launches:
        assert sum(by_id[i].batch.n_pairs + 1 for i in g) <= 45
    assert st.max_launches == 2                    # launches overlap


def test_merged_batch_matches_separate_alignment():
    """Byte-aligned merge with pad pairs: every request's slice of the
    merged results equals the request aligned on its own."""
    pool = I.random_pairs(5, 300, 50)
    cuts = [0, 7, 8, 50, 51, 120, 300]
    parts = [pool.subset(np.arange(a, b)) for a, b in zip(cuts[:-1], cuts[1:])]
    m = S.Merged(parts)
    q = np.zeros(m.q_bytes, np.uint8)
    t = np.zeros(m.t_bytes, np.uint8)
    qo = np.zeros(m.n_pairs + 1, np.int64)
    to = np.zeros(m.n_pairs + 1, np.int64)
    starts = m.fill(q, qo, t, to)
    assert qo[-1] == 4 * m.q_bytes and to[-1] == 4 * m.t_bytes
    assert np.all(np.diff(qo) >= 0) and np.all(np.diff(to) >= 0)
    got = O.align_batch(q, qo, t, to)
    for b, p in zip(parts, starts):
        want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
        for g, w in zip(got, want):
            assert np.array_equal(g[p:p + b.n_pairs], w)
