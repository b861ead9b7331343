"""Pairs at the longest supported length (65,535 bases) on every pass:
forward answers, start positions, the banded pass and the trace, each
against its oracle.  A 65,535-row target leaves room in a boundary slot for
one pair group only, so these units run one group per slot pass."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu
MAXLEN = 65535


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    salo.load()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(11)
    src = rng.integers(0, 4, MAXLEN, dtype=np.uint8)
    mut = src.copy()
    hits = rng.choice(MAXLEN, MAXLEN // 50, replace=False)
    mut[hits] = (mut[hits] + 1) & 3
    qs = [mut, src[:300].copy(), src[1000:1000 + 20000].copy(), mut[:MAXLEN]]
    ts = [src[:20000].copy(), src.copy(), src.copy(), rng.integers(0, 4, 300, dtype=np.uint8)]
    # pair 0: 65,535-base query against the first 20,000 bases of its source
    # pair 1: 300 bases against the 65,535-base source (long target)
    # pair 2: a 20,000-base window against the whole source
    # pair 3: 65,535 bases against 300 unrelated bases
    return I.from_codes(qs, ts, "maxlen")


def _say(*a):
    print("[case]", *a, flush=True)


def test_forward_and_starts(dev, batch):
    import torch
    from paper_2301_09310_amd import salo
    b = batch
    assert b.q_lens().max() == MAXLEN and b.t_lens().max() == MAXLEN
    q, qo, t, to = salo.to_device(b)
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    wst = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *want)
    for opts in ({}, {"force_int32": True}, {"cols": 32}):
        _say("maxlen forward + starts", opts)
        ans = salo.align_batch(q, qo, t, to, **opts)
        st = salo.align_starts(q, qo, t, to, ans, **opts)
        torch.cuda.synchronize()
        assert salo.error_count() == 0
        for g, w in zip(ans, want):
            assert np.array_equal(g.cpu().numpy().astype(np.int64), w)
        for g, w in zip(st, wst):
            assert np.array_equal(g.cpu().numpy().astype(np.int64), w)


@pytest.mark.parametrize("band", [0, 64, 700])
def test_banded(dev, batch, band):
    import torch
    from paper_2301_09310_amd import salo
    b = batch
    q, qo, t, to = salo.to_device(b)
    _say("maxlen banded", band)
    got = salo.align_banded(q, qo, t, to, band)
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    want = O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, band)
    for g, w in zip(got, want):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), w)


def test_trace(dev, batch):
    """Pairs 1 and 3 (short spans next to 65,535-base sequences) against the
    oracle; the 20,000 x 20,000 spans of pairs 0 and 2 need 200 MB of codes
    each, more than a wave's share of 16 GiB, so they come back as -2."""
    import torch
    from paper_2301_09310_amd import salo
    b = batch
    q, qo, t, to = salo.to_device(b)
    ans = salo.align_batch(q, qo, t, to)
    st = salo.align_starts(q, qo, t, to, ans)
    _say("maxlen trace")
    off, cig, ln = salo.align_trace(q, qo, t, to, ans, st, workspace_bytes=16 << 30)
    torch.cuda.synchronize()
    ln = ln.cpu().numpy().astype(np.int64)
    cig = cig.cpu().numpy().view(np.uint32)
    off = off.cpu().numpy()
    assert salo.error_count() == 2 and ln[0] == -2 and ln[2] == -2
    a = [x.cpu().numpy().astype(np.int64) for x in ans]
    s = [x.cpu().numpy().astype(np.int64) for x in st]
    woff, wcig, wln = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, a[0], s[0],
                                    a[1], s[1], a[2])
    for p in (1, 3):
        assert ln[p] == wln[p]
        assert np.array_equal(cig[off[p]:off[p] + ln[p]], wcig[woff[p]:woff[p] + wln[p]])


def test_forward_split_waves(dev, batch):
    """The maximum lengths with split_waves = 4: a 65,535-row unit in four
    strips of 16,384 rows (each strip's column fills half its slot)."""
    import torch
    from paper_2301_09310_amd import salo
    b = batch
    _say("maxlen forward, split waves")
    q, qo, t, to = salo.to_device(b)
    got = salo.align_batch(q, qo, t, to, split_waves=4)
    torch.cuda.synchronize()
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    for g, w in zip(got, want):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), w)
