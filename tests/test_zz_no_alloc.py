"""salo_align_batch_noalloc (the entry point that allocates nothing) called
through the C ABI, against salo_align_batch on the same inputs: two calls
in a row on one stream, the second with a smaller batch, so the second call
runs on the scratch contents the first left behind.  Both batches mix
short and long pairs (mixed workload: queries up to 10 kbp, targets up to
12 kbp), so the fixed scratch's boundary slots, plan buffers and counters
are all exercised; each answer must equal the allocating entry point's
bit for bit, and a sample is checked against the oracle.  Also: a batch
above the maximum pair count is refused and enqueues nothing."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu
SCORING = (1, -4, 6, 1)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    return salo.load()


def _call(lib, name, b, out, stream):
    from paper_2301_09310_amd import salo
    import torch
    q, qo, t, to = salo.to_device(b)
    fn = getattr(lib, name)
    st = fn(q.data_ptr(), qo.data_ptr(), t.data_ptr(), to.data_ptr(), b.n_pairs,
            salo.Scoring(*SCORING), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
            ctypes.c_void_p(stream.cuda_stream))
    assert st == 0, lib.salo_last_error().decode()
    stream.synchronize()
    res = [x[:b.n_pairs].cpu().numpy().copy() for x in out]
    del q, qo, t, to
    return res


def test_noalloc_matches_allocating_entry(lib):
    import torch
    from paper_2301_09310_amd import salo
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    big = I.mixed(3, 20_000)
    small = I.mixed(4, 3_000)
    out_na = tuple(torch.full((big.n_pairs,), 77, dtype=torch.int32, device=dev)
                   for _ in range(3))
    out_ref = tuple(torch.full((big.n_pairs,), 55, dtype=torch.int32, device=dev)
                    for _ in range(3))
    for k, b in enumerate((big, small)):
        print("[case] noalloc call %d: %d pairs, %.3e cells" % (k, b.n_pairs, b.cells()),
              flush=True)
        got = _call(lib, "salo_align_batch_noalloc", b, out_na, stream)
        want = _call(lib, "salo_align_batch", b, out_ref, stream)
        for g, w, name in zip(got, want, ("score", "q_end", "t_end")):
            bad = np.nonzero(g != w)[0]
            assert bad.size == 0, "%s differs at pair %d: noalloc %d, salo_align_batch %d" % (
                name, bad[0], g[bad[0]], w[bad[0]])
        rng = np.random.default_rng(30 + k)
        idx = np.sort(rng.choice(b.n_pairs, size=300, replace=False))
        sub = b.subset(idx)
        ora = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING)
        for g, w in zip(got, ora):
            assert np.array_equal(g[idx].astype(np.int64), w)
    # the second call's outputs past its batch are untouched
    assert bool((out_na[0][small.n_pairs:big.n_pairs] ==
                 torch.from_numpy(_call(lib, "salo_align_batch", big, out_ref, stream)[0][
                     small.n_pairs:]).to(dev)).all())


def test_noalloc_refuses_too_many_pairs(lib):
    import torch
    from paper_2301_09310_amd import salo
    dev = torch.device("cuda:0")
    n = (1 << 22) + 1
    q = torch.zeros(16, dtype=torch.uint8, device=dev)
    qo = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    out = tuple(torch.full((4,), 9, dtype=torch.int32, device=dev) for _ in range(3))
    st = lib.salo_align_batch_noalloc(q.data_ptr(), qo.data_ptr(), q.data_ptr(), qo.data_ptr(),
                                      n, salo.Scoring(*SCORING), out[0].data_ptr(),
                                      out[1].data_ptr(), out[2].data_ptr(), None)
    torch.cuda.synchronize()
    assert st == -1
    assert "maximum" in lib.salo_last_error().decode()
    assert all(bool((x == 9).all()) for x in out)
