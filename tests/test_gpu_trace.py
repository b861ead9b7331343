"""Trace pass on the GPU (salo_align_trace) against the trace oracle, bit for
bit: every pair's CIGAR runs and run count, for the GPU's own answers and
starts (themselves checked against the oracles), across scorings with and
without gap-open ties, both column counts, forced lane-group widths, long
spans, the hand-derived fixtures and a workspace too small for some pairs;
and the starts and CIGARs of every pair of the short-read batch against
the oracle's stored digests."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    salo.load()
    return torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def gpu_trace(b, scoring=(1, -4, 6, 1), workspace_bytes=1 << 30, **opts):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = salo.to_device(b)
    ans = salo.align_batch(q, qo, t, to, scoring)
    st = salo.align_starts(q, qo, t, to, ans, scoring)
    off, cig, ln = salo.align_trace(q, qo, t, to, ans, st, scoring,
                                    workspace_bytes=workspace_bytes, **opts)
    torch.cuda.synchronize()
    errors = salo.error_count()
    cpu = lambda x: x.cpu().numpy().astype(np.int64)
    return ([cpu(x) for x in ans], [cpu(x) for x in st], cpu(off),
            cig.cpu().numpy().view(np.uint32), cpu(ln), errors)


def check(b, label, scoring=(1, -4, 6, 1), **opts):
    _say(label, "pairs", b.n_pairs, "scoring", scoring, opts)
    ans, st, off, cig, ln, errors = gpu_trace(b, scoring, **opts)
    assert errors == 0
    w_ans = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, scoring)
    for g, w in zip(ans, w_ans):
        assert np.array_equal(g, w)
    w_st = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *w_ans, scoring=scoring)
    for g, w in zip(st, w_st):
        assert np.array_equal(g, w)
    woff, wcig, wln = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, w_ans[0],
                                    w_st[0], w_ans[1], w_st[1], w_ans[2], scoring)
    assert np.array_equal(off, woff)
    if not np.array_equal(ln, wln):
        p = int(np.nonzero(ln != wln)[0][0])
        raise AssertionError("%s: run count differs at pair %d: gpu %d, oracle %d"
                             % (label, p, ln[p], wln[p]))
    for p in np.nonzero(wln > 0)[0]:
        a, n = off[p], wln[p]
        if not np.array_equal(cig[a:a + n], wcig[a:a + n]):
            raise AssertionError("%s: pair %d: gpu %s, oracle %s" % (
                label, p, O.cigar_string(cig, a, n), O.cigar_string(wcig, a, n)))
    return ln


def test_plain_small(dev):
    check(I.plain_small(0, 1000), "plain_small")


@pytest.mark.parametrize("scoring", [(1, -4, 6, 1), (2, -3, 2, 1), (1, -1, 0, 1), (3, -2, 0, 2),
                                     (2, -1, 1, 1)])
def test_random_pairs(dev, scoring):
    check(I.random_pairs(41, 400, 300, min_len=0, related=0.8), "random", scoring=scoring)


@pytest.mark.parametrize("scoring", [(1, -4, 6, 1), (3, -2, 0, 2)])
def test_forced_32bit_cells(dev, scoring):
    check(I.random_pairs(44, 300, 300, min_len=0, related=0.8), "int32", scoring=scoring,
          force_int32=True)


def test_mixed_cell_kinds(dev):
    """match 16 puts the long pairs above the 16-bit bound: units of both
    kinds in one call."""
    b = I.random_pairs(45, 200, 2500, min_len=1, related=0.9)
    check(b, "mixed kinds", scoring=(16, -20, 30, 5), workspace_bytes=16 << 30)


@pytest.mark.parametrize("cols", [8, 16])
@pytest.mark.parametrize("lanes", [0, 1, 2, 4, 64])
def test_widths(dev, cols, lanes):
    # forced 4-lane groups put 16 spans of up to 600 x 600 on one wave; a
    # one-lane group walks its two pairs one after the other, wider groups
    # walk them on two lanes at once (one- and two-lane groups take spans
    # of up to 200 x 200, which fit their share of the workspace)
    longest = 200 if lanes in (1, 2) else 600
    check(I.random_pairs(42, 200, longest, min_len=1, related=0.8), "widths",
          scoring=(2, -3, 2, 1), workspace_bytes=16 << 30, cols=cols, lanes=lanes)


def test_golden_fixtures(dev):
    rows = []
    for line in open(os.path.join(HERE, "golden", "trace_examples.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            left, right = line.split("|")
            q, t, *sc = left.split()
            rows.append((q, t, tuple(int(x) for x in sc), right.split()[5]))
    for q, t, sc, cigar in rows:
        _, _, off, cig, ln, errors = gpu_trace(I.from_strings([q], [t]), sc)
        assert errors == 0
        assert O.cigar_string(cig, off[0], ln[0]) == cigar


def test_long_spans(dev):
    b = I.long_uneven(0, 2000).subset(np.arange(24))
    # a 5 kbp x 6.5 kbp span keeps 16 MB of codes: 64 GB gives every
    # resident wave room for one
    check(b, "long_uneven", workspace_bytes=64 << 30)
    a = I.anchored_long(0, 2000).subset(np.arange(24))
    check(a, "anchored_long", workspace_bytes=64 << 30)


def test_small_workspace_marks_large_pairs(dev):
    # 200 KB per wave (CUs x 8 waves at 16 columns per lane): short spans
    # fit, long ones are reported (-2) and counted; the rest are still exact
    import torch
    n_cus = torch.cuda.get_device_properties(0).multi_processor_count
    b = I.random_pairs(43, 300, 400, min_len=1, related=0.9)
    ans, st, off, cig, ln, errors = gpu_trace(b, workspace_bytes=n_cus * 8 * 200 * 1024)
    w_ans = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    w_st = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *w_ans)
    _, wcig, wln = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, w_ans[0],
                                 w_st[0], w_ans[1], w_st[1], w_ans[2])
    big = ln == -2
    assert big.any() and (~big & (wln > 0)).any() and errors == int(big.sum())
    ok = ~big
    assert np.array_equal(ln[ok], wln[ok])
    for p in np.nonzero(ok & (wln > 0))[0]:
        assert np.array_equal(cig[off[p]:off[p] + ln[p]], wcig[off[p]:off[p] + ln[p]])


def test_short_reads_full_size_sampled(dev):
    """The benchmark's short-read batch (2,000,000 pairs) end to end on the
    GPU; 300 sampled pairs against the oracles."""
    import torch
    from paper_2301_09310_amd import salo
    _say("short_reads full size")
    b = I.short_reads(0)
    q, qo, t, to = salo.to_device(b)
    ans = salo.align_batch(q, qo, t, to)
    st = salo.align_starts(q, qo, t, to, ans)
    off, cig, ln = salo.align_trace(q, qo, t, to, ans, st, workspace_bytes=4 << 30)
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    off, cig, ln = off.cpu().numpy(), cig.cpu().numpy().view(np.uint32), ln.cpu().numpy()
    idx = np.random.default_rng(6).choice(b.n_pairs, 300, replace=False)
    sub = b.subset(idx)
    w_ans = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets)
    w_st = O.start_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, *w_ans)
    woff, wcig, wln = O.trace_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets,
                                    w_ans[0], w_st[0], w_ans[1], w_st[1], w_ans[2])
    assert np.array_equal(ln[idx], wln)
    for k, p in enumerate(idx):
        assert np.array_equal(cig[off[p]:off[p] + ln[p]], wcig[woff[k]:woff[k] + wln[k]])


def test_trace_on_side_stream(dev):
    """align_trace on a stream other than the current one: the binding's own
    buffers (offsets, CIGAR arrays, workspace) are made on the launch stream
    after the current stream's work, and kept from reuse while it runs."""
    import torch
    from paper_2301_09310_amd import salo
    b = I.random_pairs(63, 400, 300, related=0.7)
    _say("trace on a side stream, pairs", b.n_pairs)
    q, qo, t, to = salo.to_device(b)
    ans = salo.align_batch(q, qo, t, to)
    st = salo.align_starts(q, qo, t, to, ans)
    side = torch.cuda.Stream()
    off, cig, ln = salo.align_trace(q, qo, t, to, ans, st, stream=side,
                                    workspace_bytes=1 << 30)
    # churn the allocator on the current stream while the side stream runs
    junk = [torch.empty(1 << 26, dtype=torch.uint8, device=dev).fill_(0xAB) for _ in range(4)]
    side.synchronize()
    torch.cuda.synchronize()
    del junk
    cpu = lambda x: x.cpu().numpy().astype(np.int64)
    w_ans = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    w_st = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *w_ans)
    woff, wcig, wln = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, w_ans[0],
                                    w_st[0], w_ans[1], w_st[1], w_ans[2])
    assert salo.error_count(side) == 0
    assert np.array_equal(cpu(off), woff)
    assert np.array_equal(cpu(ln), wln)
    g = cig.cpu().numpy().view(np.uint32)
    for p in np.nonzero(wln > 0)[0]:
        a, n = woff[p], wln[p]
        assert np.array_equal(g[a:a + n], wcig[a:a + n]), p


@pytest.mark.parametrize("workload, ws_gib", [("short_reads", 16)])
def test_every_pair_digest(dev, workload, ws_gib):
    """Start positions and CIGARs of EVERY pair of a benchmark batch
    (short_reads, 2,000,000 pairs) against the oracle's, stored as digests
    in tests/golden/trace_digests.json by tests/golden/make_trace_digests.py
    (oracle and seeded generator only), with the workspace the trace
    benchmark uses.  On a mismatch the chunk
    digests name the first 65,536-pair chunk that differs, and the oracle
    runs on its first 2,000 pairs to report the first differing pair."""
    import json
    import sys
    import torch
    from paper_2301_09310_amd import salo
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_trace_digests as D
    with open(os.path.join(HERE, "golden", "trace_digests.json")) as f:
        table = json.load(f)
    if workload not in table:
        pytest.skip("no digests stored for %s" % workload)
    want = table[workload]
    b = I.WORKLOADS[workload](0)
    assert b.sha256() == want["dataset_sha256"], "the generator changed; rerun the script"
    _say(workload, "every pair", b.n_pairs, "workspace GiB", ws_gib)
    q, qo, t, to = salo.to_device(b)
    ans = salo.align_batch(q, qo, t, to)
    st = salo.align_starts(q, qo, t, to, ans)
    off, cig, ln = salo.align_trace(q, qo, t, to, ans, st, workspace_bytes=ws_gib << 30)
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    qs, ts = (x.cpu().numpy().astype(np.int64) for x in st)
    off, cig, ln = off.cpu().numpy(), cig.cpu().numpy().view(np.uint32), ln.cpu().numpy()
    del q, qo, t, to, ans, st
    torch.cuda.empty_cache()
    runs, starts = D.packed_runs(off, cig, ln)
    got = D.trace_digests(qs, ts, ln, runs, starts, want["chunk_pairs"])
    if all(got[k] == want[k] for k in ("q_start", "t_start", "cigar_len", "cigar_runs")):
        return
    bad = next(i for i, (g, w) in enumerate(zip(got["chunks"], want["chunks"])) if g != w)
    c0 = bad * want["chunk_pairs"]
    idx = np.arange(c0, min(b.n_pairs, c0 + 2000))
    sub = b.subset(idx)
    w_ans = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets)
    w_st = O.start_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, *w_ans)
    woff, wcig, wln = O.trace_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets,
                                    w_ans[0], w_st[0], w_ans[1], w_st[1], w_ans[2])
    for k, p in enumerate(idx):
        same = (qs[p] == w_st[0][k] and ts[p] == w_st[1][k] and ln[p] == wln[k] and
                np.array_equal(cig[off[p]:off[p] + max(ln[p], 0)],
                               wcig[woff[k]:woff[k] + max(wln[k], 0)]))
        if not same:
            raise AssertionError("pair %d: gpu start (%d, %d) %s, oracle start (%d, %d) %s" % (
                p, qs[p], ts[p], O.cigar_string(cig, off[p], ln[p]), w_st[0][k], w_st[1][k],
                O.cigar_string(wcig, woff[k], wln[k])))
    raise AssertionError("chunk %d differs, but not in its first %d pairs" % (bad, len(idx)))
