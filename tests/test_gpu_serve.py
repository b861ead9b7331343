"""Served requests on the GPU: every request's result equals the oracle and
the same request aligned alone, while requests overlap on the device."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I
from paper_2301_09310_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    salo.load()
    return torch.device("cuda:0")


def test_alone_equals_mix(dev):
    import torch
    from paper_2301_09310_amd import salo
    pool = I.mixed(0, 3000)
    sizes = S.request_sizes(40, 5, max_pairs=200)
    arrivals = S.poisson_arrivals(40, 2000.0, 5)     # arrivals much faster than service
    reqs = S.split_requests(pool, sizes, arrivals)
    ex = S.GpuExecutor(n_slots=2, max_pairs=1024, max_bytes=1 << 20)
    budget = 6 * max(S.footprint_bytes(r.batch) for r in reqs)
    print("[case] serve 40 requests, budget", budget, flush=True)
    st = S.Server(ex, budget_bytes=budget).run(reqs)
    assert st.completed == 40
    assert st.max_inflight_bytes <= budget
    assert st.max_inflight >= 2
    assert max(st.launch_sizes) >= 2          # waiting requests were merged
    for r in reqs:
        b = r.batch
        want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
        q, qo, t, to = salo.to_device(b)
        alone = salo.align_batch(q, qo, t, to)
        torch.cuda.synchronize()
        for g, a, w, name in zip(r.result, alone, want, ("score", "q_end", "t_end")):
            assert np.array_equal(g, a.cpu().numpy()), (r.rid, name, "mix vs alone")
            assert np.array_equal(g.astype(np.int64), w), (r.rid, name, "mix vs oracle")


def test_served_requests_of_full_size(dev):
    """Requests of the served stream's own sizes (1..4,096 pairs of the
    mixed workload, including both extremes), arriving while others run, in
    the bench's serving configuration (per-request completion, long pairs
    on four waves): each served result equals the oracle and the same
    request aligned alone."""
    import torch
    from paper_2301_09310_amd import salo
    pool = I.mixed(0, 40_000)
    sizes = S.request_sizes(12, 21)
    sizes[0], sizes[1] = 4096, 1
    arrivals = S.poisson_arrivals(len(sizes), 400.0, 21)
    reqs = S.split_requests(pool, sizes, arrivals)
    ex = S.GpuExecutor(n_slots=3, max_pairs=1 << 15, max_bytes=32 << 20, split_waves=4)
    budget = 3 * max(S.footprint_bytes(r.batch) for r in reqs)
    print("[case] serve %d requests of %s pairs, budget %d" % (
        len(reqs), sizes.tolist(), budget), flush=True)
    st = S.Server(ex, budget_bytes=budget).run(reqs)
    assert st.completed == len(reqs)
    assert st.max_inflight_bytes <= budget
    assert st.max_inflight >= 2
    for r in reqs:
        b = r.batch
        want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
        q, qo, t, to = salo.to_device(b)
        alone = salo.align_batch(q, qo, t, to)
        torch.cuda.synchronize()
        for g, a, w, name in zip(r.result, alone, want, ("score", "q_end", "t_end")):
            assert np.array_equal(g, a.cpu().numpy()), (r.rid, name, "mix vs alone")
            assert np.array_equal(g.astype(np.int64), w), (r.rid, name, "mix vs oracle")


def test_tagged_call_counts_every_pair(dev):
    """salo_align_batch_tagged writes the answers into coherent host memory
    and counts each request's finished pairs; after the call every counter
    equals its request's size and the answers equal the oracle."""
    import torch
    from paper_2301_09310_amd import salo
    b = I.mixed(5, 3000)
    n = b.n_pairs
    rng = np.random.default_rng(6)
    tags = rng.integers(-1, 7, n).astype(np.int32)          # 7 requests, some untagged
    q, qo, t, to = salo.to_device(b)
    res = salo.HostBuffer(3 * n, np.int32)
    res.array[:] = -5
    done = salo.HostBuffer(7, np.uint32)
    done.array[:] = 0
    tag_dev = torch.from_numpy(tags).to(dev)
    print("[case] tagged call, %d pairs" % n, flush=True)
    salo.align_batch_tagged(q, qo, t, to, (1, -4, 6, 1), (res.ptr, res.ptr + 4 * n,
                                                          res.ptr + 8 * n), tag_dev, done.ptr)
    torch.cuda.synchronize()
    assert [int(x) for x in done.array] == [int((tags == k).sum()) for k in range(7)]
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    for c in range(3):
        assert np.array_equal(res.array[c * n:(c + 1) * n].astype(np.int64), want[c])
    res.free()
    done.free()
