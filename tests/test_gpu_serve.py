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
