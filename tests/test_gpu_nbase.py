"""N bases on the GPU (salo_align_batch_n, masked starts and packing)
against the oracles with the same N masks, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def n_batch(seed, n_pairs, max_len, p_n, min_len=0, only=None):
    """Random related pairs with a fraction p_n of bases turned into N
    (in both streams, or only 'q' / 't'); returns (batch, q_mask, t_mask)."""
    b = I.random_pairs(seed, n_pairs, max_len, min_len=min_len)
    rng = np.random.default_rng([seed, 77])

    def mask(total, on):
        bits = (rng.random(total) < p_n) if on else np.zeros(total, bool)
        words = np.zeros(max((total + 31) // 32, 1), np.uint32)
        idx = np.nonzero(bits)[0]
        np.bitwise_or.at(words, idx >> 5, (np.uint32(1) << (idx & 31).astype(np.uint32)))
        return words
    qm = mask(int(b.q_offsets[-1]), only in (None, "q"))
    tm = mask(int(b.t_offsets[-1]), only in (None, "t"))
    return b, qm, tm


def gpu_run(b, qm, tm, scoring=(1, -4, 6, 1), starts=True, **opts):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = salo.to_device(b)
    qmd = torch.from_numpy(qm.view(np.int32)).cuda()
    tmd = torch.from_numpy(tm.view(np.int32)).cuda()
    ans = salo.align_batch(q, qo, t, to, scoring, q_nmask=qmd, t_nmask=tmd, **opts)
    st = None
    if starts:
        st = salo.align_starts(q, qo, t, to, ans, scoring, q_nmask=qmd, t_nmask=tmd,
                               **{k: v for k, v in opts.items() if k != "mode"})
    torch.cuda.synchronize()
    ans = tuple(x.cpu().numpy().astype(np.int64) for x in ans)
    st = None if st is None else tuple(x.cpu().numpy().astype(np.int64) for x in st)
    return ans, st


def check(b, qm, tm, label, scoring=(1, -4, 6, 1), starts=True, **opts):
    ans, st = gpu_run(b, qm, tm, scoring, starts, **opts)
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, scoring,
                         q_nmask=qm, t_nmask=tm)
    for g, w, name in zip(ans, want, ("score", "q_end", "t_end")):
        bad = np.nonzero(g != w)[0]
        assert bad.size == 0, "%s: %s differs at pair %d: gpu %d oracle %d" % (
            label, name, bad[0], g[bad[0]], w[bad[0]])
    if starts:
        ws = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *want, scoring=scoring,
                           q_nmask=qm, t_nmask=tm)
        for g, w, name in zip(st, ws, ("q_start", "t_start")):
            assert np.array_equal(g, w), (label, name)


@pytest.mark.parametrize("scoring", [(1, -4, 6, 1), (2, -3, 5, 2), (1, 0, 0, 0), (200, -100, 50, 7)])
def test_scorings(dev, scoring):
    b, qm, tm = n_batch(51, 600, 400, 0.03)
    for opts in ({}, {"force_int32": True}, {"mode": "plain", "lanes": 4, "cols": 16}):
        _say("N masks scoring", scoring, opts)
        check(b, qm, tm, "scoring %s %s" % (scoring, opts), scoring,
              starts=opts.get("mode") != "plain", **opts)


@pytest.mark.parametrize("only", ["q", "t"])
def test_mask_on_one_side(dev, only):
    b, qm, tm = n_batch(52, 400, 300, 0.05, only=only)
    _say("N only in", only)
    check(b, qm, tm, "only " + only)


@pytest.mark.parametrize("cols", [8, 16, 32])
@pytest.mark.parametrize("lanes", [1, 4, 16, 64])
def test_forced_widths(dev, lanes, cols):
    b, qm, tm = n_batch(53, 250, 700, 0.02)
    _say("N masks lanes", lanes, "cols", cols)
    check(b, qm, tm, "lanes %d cols %d" % (lanes, cols), lanes=lanes, cols=cols)


def test_dense_n(dev):
    b, qm, tm = n_batch(54, 300, 200, 0.5)
    _say("half the bases N")
    check(b, qm, tm, "dense N")


def test_long_pairs_with_n(dev):
    b, qm, tm = n_batch(55, 60, 5000, 0.01, min_len=1000)
    _say("long pairs with N")
    check(b, qm, tm, "long N")


def test_pack_n_mask_then_align(dev):
    """Characters with N (and n) packed on the GPU with an N mask, forward
    and reverse-complemented, equal the packing oracle; aligning the packed
    streams with their masks equals the alignment oracle."""
    import torch
    from paper_2301_09310_amd import salo
    rng = np.random.default_rng(56)
    letters = np.frombuffer(b"ACGTNacgtn", np.uint8)
    for rc in (False, True):
        q_lens = rng.integers(0, 300, 700)
        t_lens = rng.integers(0, 400, 700)
        qo = np.concatenate([[0], np.cumsum(q_lens)]).astype(np.int64)
        to = np.concatenate([[0], np.cumsum(t_lens)]).astype(np.int64)
        qc = letters[rng.choice(10, int(qo[-1]), p=[.23, .23, .23, .23, .02, .0125, .0125, .0125, .0125, .01])]
        tc = letters[rng.choice(10, int(to[-1]), p=[.23, .23, .23, .23, .02, .0125, .0125, .0125, .0125, .01])]
        qc[::997] = ord("X")                          # a few invalid characters
        dq = torch.from_numpy(qc).cuda()
        dt = torch.from_numpy(tc).cuda()
        dqo, dto = torch.from_numpy(qo).cuda(), torch.from_numpy(to).cuda()
        qmask = torch.full(((qc.size + 31) // 32,), -1, dtype=torch.int32, device="cuda")
        tmask = torch.full(((tc.size + 31) // 32,), -1, dtype=torch.int32, device="cuda")
        inv = torch.zeros(1, dtype=torch.int64, device="cuda")
        _say("pack with N mask, revcomp", rc)
        qp = salo.pack_bases(dq, dqo, revcomp=rc, n_mask=qmask, invalid=inv)
        tp = salo.pack_bases(dt, dto, revcomp=rc, n_mask=tmask)
        ans = salo.align_batch(qp, dqo, tp, dto, q_nmask=qmask, t_nmask=tmask)
        torch.cuda.synchronize()
        wq, wbad, wqm = O.pack(qc, qo, revcomp=rc, nmask=True)
        wt, _, wtm = O.pack(tc, to, revcomp=rc, nmask=True)
        assert np.array_equal(qp.cpu().numpy()[: wq.size], wq)
        assert np.array_equal(tp.cpu().numpy()[: wt.size], wt)
        assert np.array_equal(qmask.cpu().numpy().view(np.uint32), wqm)
        assert np.array_equal(tmask.cpu().numpy().view(np.uint32), wtm)
        assert int(inv.item()) == wbad
        want = O.align_batch(wq, qo, wt, to, q_nmask=wqm, t_nmask=wtm)
        for g, w in zip(ans, want):
            assert np.array_equal(g.cpu().numpy().astype(np.int64), w)


def test_short_reads_with_n_every_pair_digest(dev):
    """EVERY pair of the benchmark's short-read batch with 1% of the bases of
    both streams marked N (inputs.random_n_masks, the masks bench.py
    --n-fraction 0.01 uses) against the oracle's answers, stored as digests
    in tests/golden/n_digests.json by tests/golden/make_n_digests.py (oracle
    and seeded generators only).  On a mismatch the chunk digests name the
    first 65,536-pair chunk that differs (the other tests of this file
    compare pair by pair)."""
    import hashlib
    import json
    import os
    import torch
    from paper_2301_09310_amd import salo
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "n_digests.json")) as f:
        want = json.load(f)["short_reads_n001"]
    b = I.short_reads(0)
    assert b.sha256() == want["dataset_sha256"], "the generator changed; rerun the script"
    qm, tm = I.random_n_masks(int(b.q_offsets[-1]), int(b.t_offsets[-1]),
                              want["n_fraction"], want["n_seed"])
    sha = lambda a, dt: hashlib.sha256(np.ascontiguousarray(a, dtype=dt).tobytes()).hexdigest()
    assert sha(qm, "<u4") == want["q_nmask"] and sha(tm, "<u4") == want["t_nmask"]
    _say("short_reads with N, every pair", b.n_pairs)
    q, qo, t, to = salo.to_device(b)
    qmd = torch.from_numpy(qm.view(np.int32)).cuda()
    tmd = torch.from_numpy(tm.view(np.int32)).cuda()
    out = salo.align_batch(q, qo, t, to, q_nmask=qmd, t_nmask=tmd)
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    got = tuple(x.cpu().numpy() for x in out)
    del q, qo, t, to, out, qmd, tmd
    torch.cuda.empty_cache()
    if all(sha(g, "<i4") == want[k] for g, k in zip(got, ("score", "q_end", "t_end"))):
        return
    chunk = want["chunk_pairs"]
    for c, wd in enumerate(want["chunks"]):
        h = hashlib.sha256()
        for a in got:
            h.update(np.ascontiguousarray(a[c * chunk:(c + 1) * chunk], dtype="<i4").tobytes())
        if h.hexdigest() != wd:
            break
    raise AssertionError("chunk %d (pairs %d..) differs from the oracle's digest"
                         % (c, c * chunk))
