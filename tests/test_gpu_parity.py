"""GPU parity: the HIP library against the CPU oracle, bit-exact on every
(score, q_end, t_end) -- the operation is integer-valued, so the tolerance
is zero.  Every call goes through the C ABI (salo_align_batch_ex).

Each test prints the case (workload, seed, options) before its GPU step."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu

SCORING = (1, -4, 6, 1)
PLAIN_VARIANTS = [(1, 16), (2, 16), (4, 16), (8, 16), (16, 16), (32, 16), (64, 16),
                  (2, 8), (4, 8), (8, 8), (16, 8), (1, 32), (2, 32), (8, 32), (64, 8)]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    salo.load()          # raises if the library is missing: no fallback
    return torch.device("cuda:0")


def gpu_align(batch, scoring=SCORING, **opts):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = salo.to_device(batch)
    out = salo.align_batch(q, qo, t, to, scoring, **opts)
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy().astype(np.int64) for x in out)


def oracle_align(batch, scoring=SCORING):
    return O.align_batch(batch.q_seqs, batch.q_offsets, batch.t_seqs, batch.t_offsets,
                         scoring)


def assert_same(batch, got, want, label):
    names = ("score", "q_end", "t_end")
    for k in range(3):
        bad = np.nonzero(got[k] != want[k])[0]
        if bad.size:
            p = int(bad[0])
            q, t = batch.pair_strings(p) if batch.q_lens()[p] < 400 else ("...", "...")
            pytest.fail("%s: %d mismatches in %s; first pair %d (m=%d n=%d): gpu %s oracle %s"
                        " q=%s t=%s" % (label, bad.size, names[k], p, batch.q_lens()[p],
                                        batch.t_lens()[p],
                                        tuple(int(g[p]) for g in got),
                                        tuple(int(w[p]) for w in want), q, t))


def test_plain_small_default(dev):
    b = I.plain_small()
    _say("plain_small seed 0, default options")
    got = gpu_align(b)
    assert_same(b, got, oracle_align(b), "plain_small")


@pytest.mark.parametrize("lanes,cols", PLAIN_VARIANTS)
def test_random_pairs_every_variant(dev, lanes, cols):
    b = I.random_pairs(11, 600, 300)
    want = oracle_align(b)
    _say("random_pairs seed 11 plain lanes=%d cols=%d" % (lanes, cols))
    assert_same(b, gpu_align(b, mode="plain", lanes=lanes, cols=cols), want,
                "lanes=%d cols=%d" % (lanes, cols))
    _say("random_pairs seed 11 plain lanes=%d cols=%d int32" % (lanes, cols))
    assert_same(b, gpu_align(b, mode="plain", lanes=lanes, cols=cols, force_int32=True),
                want, "lanes=%d cols=%d int32" % (lanes, cols))


@pytest.mark.parametrize("scoring", [(1, -4, 6, 1), (2, -3, 5, 2), (1, -1, 1, 1),
                                     (3, 0, 2, 1), (1, -2, 0, 1), (5, -4, 3, 0),
                                     (1, -4, 0, 0), (200, -100, 50, 7), (7, -300, 12, 3),
                                     (8, -12, 10, 2), (16, -20, 30, 5), (1, 0, 0, 0),
                                     (2, -2048, 2046, 1)])
def test_scorings(dev, scoring):
    """Scorings whose values fit a binary16 row table (one byte each) run in
    binary16 cells where the score bound allows; the others, and every
    scoring with binary16 switched off, in 16-bit integer or 32-bit cells."""
    b = I.random_pairs(21, 400, 200)
    want = oracle_align(b, scoring)
    for lanes, cols in [(4, 16), (16, 8)]:
        for no_f16 in (False, True):
            _say("random_pairs seed 21 scoring", scoring, "lanes", lanes, "cols", cols,
                 "no_f16", no_f16)
            assert_same(b, gpu_align(b, scoring, mode="plain", lanes=lanes, cols=cols,
                                     no_f16=no_f16), want,
                        "scoring %s no_f16=%s" % (scoring, no_f16))
    _say("random_pairs seed 21 scoring", scoring, "persistent")
    assert_same(b, gpu_align(b, scoring), want, "scoring %s persistent" % (scoring,))


def test_binary16_limit_edge(dev):
    """Best scores at and just past 2048, the largest integer up to which
    binary16 cells are exact (match * min(m, n) <= 2048 keeps a pair in
    binary16 cells; one more base moves it to 16-bit integer cells)."""
    rng = np.random.default_rng(78)
    qs, ts = [], []
    for match, mns in ((1, (2047, 2048, 2049)), (4, (511, 512, 513))):
        for mn in mns:
            base = rng.integers(0, 4, mn).astype(np.uint8)
            qs.append(base)
            ts.append(base.copy())
            mut = base.copy()
            mut[rng.choice(mn, 3, replace=False)] ^= 2
            qs.append(base)
            ts.append(np.concatenate([mut, rng.integers(0, 4, 5).astype(np.uint8)]))
    b = I.from_codes(qs, ts, "binary16_limit")
    for match in (1, 4):
        sc = (match, -4, 6, 1)
        want = oracle_align(b, sc)
        for opts in ({"mode": "plain", "lanes": 64, "cols": 16}, {"mode": "persistent"},
                     {"mode": "persistent", "no_f16": True}):
            _say("binary16 limit scoring", sc, opts)
            assert_same(b, gpu_align(b, sc, **opts), want, "binary16 limit %s %s" % (sc, opts))


def _edge_batch():
    rng = np.random.default_rng(5)
    qs, ts = [], []
    # empty and tiny
    for m, n in [(0, 0), (0, 5), (5, 0), (1, 1), (1, 7), (7, 1), (2, 2)]:
        qs.append(rng.integers(0, 4, m, dtype=np.uint8))
        ts.append(rng.integers(0, 4, n, dtype=np.uint8))
    # lengths around chunk widths (lanes*cols for several variants) and rows
    for L in [7, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257,
              1023, 1024, 1025]:
        t = rng.integers(0, 4, L + 3, dtype=np.uint8)
        qs.append(t[2:2 + L].copy())
        ts.append(t)
        qs.append(rng.integers(0, 4, L, dtype=np.uint8))
        ts.append(rng.integers(0, 4, max(1, L // 3), dtype=np.uint8))
    # tie-heavy: homopolymers and two-letter alphabets
    for L in [5, 40, 150]:
        qs.append(np.zeros(L, np.uint8)); ts.append(np.zeros(L + 7, np.uint8))
        qs.append(rng.integers(0, 2, L, dtype=np.uint8))
        ts.append(rng.integers(0, 2, 2 * L, dtype=np.uint8))
    # very uneven shapes
    qs.append(rng.integers(0, 4, 1500, dtype=np.uint8)); ts.append(rng.integers(0, 4, 9, dtype=np.uint8))
    qs.append(rng.integers(0, 4, 9, dtype=np.uint8)); ts.append(rng.integers(0, 4, 3000, dtype=np.uint8))
    # identical long strings (score = length)
    s = rng.integers(0, 4, 2000, dtype=np.uint8)
    qs.append(s.copy()); ts.append(s.copy())
    return I.from_codes(qs, ts)


def test_edge_cases(dev):
    b = _edge_batch()
    want = oracle_align(b)
    assert want[0][-1] == 2000
    for lanes, cols in PLAIN_VARIANTS:
        _say("edge cases lanes=%d cols=%d" % (lanes, cols))
        assert_same(b, gpu_align(b, mode="plain", lanes=lanes, cols=cols), want,
                    "edges lanes=%d cols=%d" % (lanes, cols))
    _say("edge cases default")
    assert_same(b, gpu_align(b), want, "edges default")


def test_int32_forced_by_score_bound(dev):
    """match=16 puts long pairs above the 16-bit bound (16*(min+1) > 32767)."""
    b = I.long_uneven(0, 60)
    sc = (16, -20, 30, 5)
    want = oracle_align(b, sc)
    assert int(want[0].max()) > 32767
    _say("long_uneven 60 pairs scoring", sc)
    assert_same(b, gpu_align(b, sc), want, "int32 by bound")


def test_packed_limit_edge(dev):
    """Scores right at the largest 16-bit cell value (0x7BFF), where the
    half-precision maximum still orders cells exactly, and one base past
    it, where the pair moves to 32-bit cells.  With match=16 and
    mismatch=-1 a pair with min(m, n) = 1982 has 16*1983+1 = 31729 <= 31743
    (16-bit) and min(m, n) = 1983 has 31745 (32-bit)."""
    rng = np.random.default_rng(77)
    qs, ts = [], []
    for mn in (1982, 1983):
        base = rng.integers(0, 4, mn).astype(np.uint8)
        qs.append(base)
        ts.append(base.copy())                       # perfect match: score 16*mn
        mut = base.copy()
        mut[rng.choice(mn, 4, replace=False)] ^= 1   # four substitutions
        qs.append(base)
        ts.append(mut)
        qs.append(base[: mn - 7])                    # query ends inside the target
        ts.append(np.concatenate([rng.integers(0, 4, 9).astype(np.uint8), base]))
    b = I.from_codes(qs, ts, "packed_limit")
    sc = (16, -1, 6, 1)
    want = oracle_align(b, sc)
    assert int(want[0][0]) == 16 * 1982 and int(want[0][3]) == 16 * 1983
    for mode in ("plain", "persistent"):
        _say("packed limit edge mode", mode)
        assert_same(b, gpu_align(b, sc, mode=mode), want, "packed limit " + mode)


def test_invalid_pairs_are_flagged(dev):
    import torch
    from paper_2301_09310_amd import salo
    b = I.random_pairs(3, 40, 50)
    qo = b.q_offsets.copy()
    qo[10] = qo[11] + 5              # pair 10 gets a negative length (pair 9 a longer one)
    to = b.t_offsets.copy()
    to[21] = to[20] + 70000          # pair 20 gets a target above 65535 bases, 21 a negative one
    bad = I.Batch(b.q_seqs, qo, b.t_seqs, to)
    salo.error_count()               # reset
    _say("invalid pairs")
    got = gpu_align(bad)
    for p in (10, 20, 21):
        assert got[0][p] == -1 and got[1][p] == -1 and got[2][p] == -1
    assert salo.error_count() == 3
    want = oracle_align(b)
    ok = [p for p in range(40) if p not in (9, 10, 20, 21)]
    for k in range(3):
        assert np.array_equal(got[k][ok], want[k][ok])


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("cols", [8, 16, 32])
def test_persistent_forced_widths(dev, lanes, cols):
    b = _edge_batch()
    want = oracle_align(b)
    _say("edge cases persistent lanes=%d cols=%d" % (lanes, cols))
    assert_same(b, gpu_align(b, mode="persistent", lanes=lanes, cols=cols), want,
                "persistent lanes=%d cols=%d" % (lanes, cols))


def _uneven_rows_batch(seed):
    """Pairs of one query-length bin whose target lengths differ inside a
    unit: lengths a few rows apart (one sort level, so they share units:
    the steps free of the per-pair row test end at the shortest, at any
    remainder mod 4), lengths far apart (mixed in the plain kernel's
    consecutive units), and empty and one-row targets.  Half the queries
    are the target's last bases, so the best cell sits in a pair's last
    rows, right where the row test starts to matter."""
    rng = np.random.default_rng(seed)
    qs, ts = [], []
    for p in range(1200):
        m = int(rng.integers(100, 131))
        n = int(rng.choice([597, 598, 599, 600, 601, 602, 603, 604])) if p % 5 else \
            int(rng.choice([0, 1, 3, 40, 250, 900]))
        t = rng.integers(0, 4, n, dtype=np.uint8)
        if p % 2 == 0 and n >= m:
            q = t[n - m:].copy()
            q[rng.integers(0, m, 3)] = rng.integers(0, 4, 3)     # a few substitutions
        else:
            q = rng.integers(0, 4, m, dtype=np.uint8)
        qs.append(q)
        ts.append(t)
    return I.from_codes(qs, ts, "uneven_rows")


@pytest.mark.parametrize("kw", [{}, {"mode": "plain", "lanes": 4, "cols": 16},
                                {"mode": "plain", "lanes": 2, "cols": 32},
                                {"mode": "persistent", "lanes": 8, "cols": 8},
                                {"mode": "persistent", "lanes": 64, "cols": 16},
                                {"mode": "persistent", "no_f16": True},
                                {"mode": "persistent", "force_int32": True}])
def test_pairs_of_uneven_rows_in_one_unit(dev, kw):
    b = _uneven_rows_batch(17)
    want = oracle_align(b)
    _say("uneven rows in one unit", kw)
    assert_same(b, gpu_align(b, **kw), want, "uneven rows %s" % kw)


def test_modes_agree_on_mixed_lengths(dev):
    """Plain and persistent (binned, sorted) runs give identical outputs."""
    b = I.random_pairs(31, 3000, 1500, related=0.7)
    want = oracle_align(b)
    for mode, kw in [("persistent", {}), ("persistent", {"cols": 8}),
                     ("plain", {"lanes": 8, "cols": 16}), ("auto", {}),
                     ("persistent", {"force_int32": True})]:
        _say("random_pairs seed 31 mode", mode, kw)
        assert_same(b, gpu_align(b, mode=mode, **kw), want, "mode %s %s" % (mode, kw))


def test_short_reads_subset(dev):
    """200,000 pairs of the short-read workload, every pair checked."""
    b = I.short_reads(0, 200_000)
    want = oracle_align(b)
    _say("short_reads 200k pairs default")
    assert_same(b, gpu_align(b), want, "short_reads 200k")
    _say("short_reads 200k pairs plain")
    assert_same(b, gpu_align(b, mode="plain"), want, "short_reads 200k plain")


def test_long_uneven_sample(dev):
    b = I.long_uneven(0, 2000)
    want = oracle_align(b)
    _say("long_uneven 2000 pairs default")
    assert_same(b, gpu_align(b), want, "long_uneven 2000")


def test_mixed_sample(dev):
    b = I.mixed(0, 6000)
    want = oracle_align(b)
    _say("mixed 6000 pairs default")
    assert_same(b, gpu_align(b), want, "mixed 6000")


def test_bin_table_does_not_change_results(dev):
    from paper_2301_09310_amd import salo
    b = I.random_pairs(41, 2000, 2500, related=0.6)
    want = oracle_align(b)
    before = salo.get_bins()
    try:
        for table in ([(300, 1, 64), (65535, 1, 1), (65535, 0, 2)],
                      [(50, 1, 8), (100, 1, 1), (400, 1, 32), (65535, 1, 4), (500, 0, 64),
                       (65535, 0, 1)],
                      # a column count per bin: one persistent launch per class
                      [(64, 1, 4, 8), (200, 1, 2, 32), (800, 1, 16, 16), (65535, 1, 64, 8),
                       (300, 0, 8, 32), (65535, 0, 32, 8)],
                      [(128, 1, 1, 32), (1024, 1, 8, 8), (65535, 1, 32, 32),
                       (65535, 0, 4, 16)]):
            salo.set_bins(table)
            _say("bin table", table)
            assert_same(b, gpu_align(b), want, "table %s" % (table,))
            assert_same(b, gpu_align(b, force_int32=True), want, "table %s int32" % (table,))
    finally:
        salo.set_bins(None)
    assert salo.get_bins() == before


def test_bin_boundaries_with_both_cell_widths(dev):
    """match=16 sends long pairs to 32-bit bins and short ones to 16-bit bins,
    so units at the end of one bin sit next to pairs of a very different
    length in the processing order."""
    b = I.random_pairs(43, 400, 6000, related=0.6)
    sc = (16, -20, 30, 5)
    want = oracle_align(b, sc)
    _say("random_pairs seed 43, lengths to 6000, scoring", sc)
    assert_same(b, gpu_align(b, sc), want, "both widths")
    assert_same(b, gpu_align(b, sc, cols=8), want, "both widths cols 8")


def test_graph_capture_replays(dev):
    """Plan + persistent launches captured in a HIP graph: every replay, with
    eager work and synchronisations in between, equals the eager result."""
    import torch
    from paper_2301_09310_amd import salo
    b1 = I.random_pairs(51, 3000, 700, related=0.6)
    # same shapes, other content: swap A<->C and G<->T in every query
    b2 = I.Batch(b1.q_seqs ^ np.uint8(0x55), b1.q_offsets, b1.t_seqs, b1.t_offsets)
    want1, want2 = oracle_align(b1), oracle_align(b2)
    s = torch.cuda.Stream()
    q, qo, t, to = salo.to_device(b1)
    out = tuple(torch.empty(b1.n_pairs, dtype=torch.int32, device="cuda") for _ in range(3))
    with torch.cuda.stream(s):
        salo.reserve(b1.n_pairs, stream=s)
        salo.align_batch(q, qo, t, to, out=out, stream=s)     # warm-up on the capture stream
    s.synchronize()
    _say("graph capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        salo.align_batch(q, qo, t, to, out=out, stream=s)
    for rep in range(4):
        src = b1 if rep % 2 == 0 else b2
        d = salo.to_device(src)
        for x, y in zip((q, qo, t, to), d):
            x.copy_(y)
        for o in out:
            o.fill_(-7)                                      # eager work between replays
        torch.cuda.synchronize()
        _say("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        got = tuple(x.cpu().numpy().astype(np.int64) for x in out)
        assert_same(src, got, want1 if rep % 2 == 0 else want2, "replay %d" % rep)


def test_graph_capture_all_passes(dev):
    """Forward, start, trace and banded calls captured together in one HIP
    graph: every replay, on alternating inputs of the same shapes with eager
    work in between, equals the oracles."""
    import torch
    from paper_2301_09310_amd import salo
    b1 = I.random_pairs(52, 1500, 500, related=0.7)
    b2 = I.Batch(b1.q_seqs ^ np.uint8(0x55), b1.q_offsets, b1.t_seqs, b1.t_offsets)
    wants = []
    for b in (b1, b2):
        a = oracle_align(b)
        st = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *a)
        tr = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, a[0], st[0], a[1],
                           st[1], a[2])
        bd = O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, 40)
        wants.append((a, st, tr, bd))
    n = b1.n_pairs
    s = torch.cuda.Stream()
    q, qo, t, to = salo.to_device(b1)
    i32 = lambda: torch.empty(n, dtype=torch.int32, device="cuda")
    ans, sts, band = (i32(), i32(), i32()), (i32(), i32()), (i32(), i32(), i32())
    cig_off = salo.cigar_offsets(qo, to)
    cig = torch.zeros(int(cig_off[-1].item()), dtype=torch.int32, device="cuda")
    cig_len = i32()
    ws = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")

    def calls():
        salo.align_batch(q, qo, t, to, out=ans, stream=s)
        salo.align_starts(q, qo, t, to, ans, out=sts, stream=s)
        salo.align_trace(q, qo, t, to, ans, sts, cig_off=cig_off, workspace=ws,
                         out=(cig, cig_len), stream=s)
        salo.align_banded(q, qo, t, to, 40, out=band, stream=s)
    with torch.cuda.stream(s):
        salo.reserve(n, stream=s)
        calls()                                        # warm-up on the capture stream
    s.synchronize()
    assert salo.error_count(s) == 0
    _say("graph capture of all passes")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        calls()
    off = cig_off.cpu().numpy()
    for rep in range(4):
        src = b1 if rep % 2 == 0 else b2
        a, st, (woff, wcig, wln), bd = wants[rep % 2]
        for x, y in zip((q, qo, t, to), salo.to_device(src)):
            x.copy_(y)
        for o in ans + sts + band + (cig_len,):
            o.fill_(-7)                                # eager work between replays
        torch.cuda.synchronize()
        _say("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        cpu = lambda x: x.cpu().numpy().astype(np.int64)
        for got, want in ((ans, a), (sts, st), (band, bd)):
            for x, y in zip(got, want):
                assert np.array_equal(cpu(x), y), "replay %d" % rep
        ln = cpu(cig_len)
        assert np.array_equal(ln, wln), "replay %d" % rep
        cg = cig.cpu().numpy().view(np.uint32)
        for p in np.nonzero(wln > 0)[0]:
            assert np.array_equal(cg[off[p]:off[p] + ln[p]], wcig[woff[p]:woff[p] + wln[p]])


def test_capture_on_unreserved_stream_is_refused(dev):
    """A first call on a stream made under graph capture cannot create its
    workspace: it returns SALO_ERR_CAPTURE and enqueues nothing, and an
    eager call on the same stream afterwards works and is exact."""
    import torch
    from paper_2301_09310_amd import salo
    b = I.random_pairs(53, 800, 400, related=0.6)
    want = oracle_align(b)
    s = torch.cuda.Stream()
    q, qo, t, to = salo.to_device(b)
    out = tuple(torch.full((b.n_pairs,), -9, dtype=torch.int32, device="cuda")
                for _ in range(3))
    torch.cuda.synchronize()
    _say("capture on an unreserved stream")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(salo.SaloError) as err:
        with torch.cuda.graph(g, stream=s):
            salo.align_batch(q, qo, t, to, out=out, stream=s)
    assert err.value.status == -4
    torch.cuda.synchronize()
    assert all(bool((x == -9).all()) for x in out)
    with torch.cuda.stream(s):
        salo.align_batch(q, qo, t, to, out=out, stream=s)
    s.synchronize()
    got = tuple(x.cpu().numpy().astype(np.int64) for x in out)
    assert_same(b, got, want, "eager after a refused capture")


def test_growth_after_capture_keeps_the_graph_valid(dev):
    """A graph captured on a stream keeps working after a larger eager call
    on that stream has grown the workspace (the captured buffers are kept,
    not freed)."""
    import torch
    from paper_2301_09310_amd import salo
    small = I.random_pairs(54, 1000, 600, related=0.6)
    big = I.random_pairs(55, 30000, 300, related=0.6)
    want_s, want_b = oracle_align(small), oracle_align(big)
    s = torch.cuda.Stream()
    q, qo, t, to = salo.to_device(small)
    out = tuple(torch.empty(small.n_pairs, dtype=torch.int32, device="cuda") for _ in range(3))
    with torch.cuda.stream(s):
        salo.reserve(small.n_pairs, stream=s)
        salo.align_batch(q, qo, t, to, out=out, stream=s)
    s.synchronize()
    _say("capture, then grow the workspace with a larger eager call")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        salo.align_batch(q, qo, t, to, out=out, stream=s)
    qb, qob, tb, tob = salo.to_device(big)
    with torch.cuda.stream(s):
        ob = salo.align_batch(qb, qob, tb, tob, stream=s)
    s.synchronize()
    assert_same(big, tuple(x.cpu().numpy().astype(np.int64) for x in ob), want_b, "grown")
    for rep in range(3):
        for o in out:
            o.fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = tuple(x.cpu().numpy().astype(np.int64) for x in out)
        assert_same(small, got, want_s, "replay %d after growth" % rep)


@pytest.mark.parametrize("case", ["long_uneven", "mixed", "random", "edges"])
def test_split_waves_match_the_oracle(dev, case):
    """split_waves = 4: the 64-lane bins' units run on four waves each, one
    strip of target rows per wave; every answer equals the oracle's
    (strip boundaries inside alignments, pairs of one unit with different
    lengths, units too short to split, 32-bit cells)."""
    if case == "long_uneven":
        b = I.long_uneven(0, 600)
    elif case == "mixed":
        b = I.mixed(2, 4000)
    elif case == "random":
        b = I.random_pairs(57, 800, 3000, min_len=200, related=0.7)
    else:
        # identical strings (the best cell is the last row), one long pair
        # beside a short one, rows just above and below the split threshold
        rng = np.random.default_rng(58)
        qs, ts = [], []
        for n in (1024, 1023, 1025, 2048, 2047, 4096, 5000, 257, 1100, 3333):
            t = rng.integers(0, 4, n).astype(np.uint8)
            qs.append(t.copy())
            ts.append(t)
        for m, n in ((3000, 5000), (2500, 400), (1200, 9000), (5000, 1030)):
            t = rng.integers(0, 4, n).astype(np.uint8)
            q = rng.integers(0, 4, m).astype(np.uint8)
            k = min(m, n) // 2
            q[:k] = t[n - k:]
            qs.append(q)
            ts.append(t)
        b = I.from_codes(qs, ts)
    want = oracle_align(b)
    _say("split waves", case, b.n_pairs)
    assert_same(b, gpu_align(b, split_waves=4), want, "split %s" % case)
    if case == "random":
        assert_same(b, gpu_align(b, split_waves=4, force_int32=True), want, "split int32")
        assert_same(b, gpu_align(b, split_waves=4, no_f16=True), want, "split u16")
