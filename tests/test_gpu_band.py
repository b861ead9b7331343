"""Banded alignment on the GPU (salo_align_batch_banded) against the banded
oracle (Eq. 1 restricted to |i - j| <= band), bit for bit: scores and end
positions, over band widths from 0 to wider than every pair, every lane-group
width and column count, every cell type, the boundary ring of long targets,
and every pair of the anchored long workload at the benchmark's launch
configuration (against the band oracle's stored digests)."""
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


def gpu_banded(b, band, scoring=(1, -4, 6, 1), **opts):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = salo.to_device(b)
    out = salo.align_banded(q, qo, t, to, band, scoring, **opts)
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    return tuple(x.cpu().numpy().astype(np.int64) for x in out)


def check(b, band, label, scoring=(1, -4, 6, 1), **opts):
    _say(label, "pairs", b.n_pairs, "band", band, "scoring", scoring, opts)
    got = gpu_banded(b, band, scoring, **opts)
    want = O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, band, scoring)
    for name, g, w in zip(("score", "q_end", "t_end"), got, want):
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            p = int(bad[0])
            raise AssertionError(
                "%s: %s differs at %d of %d pairs; first pair %d (m=%d n=%d): gpu %s, oracle %s"
                % (label, name, bad.size, b.n_pairs, p, b.q_lens()[p], b.t_lens()[p],
                   tuple(int(x[p]) for x in got), tuple(int(x[p]) for x in want)))
    return got


@pytest.mark.parametrize("band", [0, 1, 3, 10, 40, 100, 250])
def test_plain_small(dev, band):
    check(I.plain_small(0, 1000), band, "plain_small")


@pytest.mark.parametrize("band", [0, 1, 7, 33, 129])
def test_random_lengths_with_empty_pairs(dev, band):
    check(I.random_pairs(21, 400, 300, min_len=0, related=0.7), band, "random")


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("cols", [8, 16, 32])
def test_every_width(dev, lanes, cols):
    b = I.random_pairs(22, 160, 420, min_len=1, related=0.8)
    for band in (5, 70):
        check(b, band, "width", lanes=lanes, cols=cols)


@pytest.mark.parametrize("opts", [dict(force_int32=True), dict(no_f16=True), dict()])
@pytest.mark.parametrize("scoring", [(1, -4, 6, 1), (2, -3, 5, 2), (1, -1, 0, 1), (3, -2, 2, 0)])
def test_cell_types_and_scorings(dev, opts, scoring):
    b = I.random_pairs(23, 200, 350, min_len=1, related=0.8)
    check(b, 24, "cells", scoring=scoring, **opts)


def test_wide_band_is_the_unbanded_answer(dev):
    import torch
    from paper_2301_09310_amd import salo
    b = I.random_pairs(24, 300, 500, min_len=0, related=0.6)
    got = check(b, 65535, "wide")
    q, qo, t, to = salo.to_device(b)
    ref = salo.align_batch(q, qo, t, to)
    torch.cuda.synchronize()
    for g, r in zip(got, ref):
        assert np.array_equal(g, r.cpu().numpy().astype(np.int64))


def test_ring_wraps_on_long_targets(dev):
    # targets far longer than the ring (2w+2 rows, rounded up to a power of
    # two): the boundary rows of every chunk wrap around the slot
    b = I.anchored_long(3, 120)
    for band, lanes in ((3, 1), (20, 2), (100, 0), (100, 8)):
        check(b, band, "ring", lanes=lanes)


def test_long_pairs_in_one_unit_need_several_slot_passes(dev):
    # a band wider than half the slot's rows per group forces fewer groups
    # per pass: 64 one-lane groups cannot all hold 8192 rows
    b = I.anchored_long(4, 64)
    check(b, 3000, "passes", lanes=1, cols=8)


def test_anchored_long_full_size_sampled(dev):
    """The benchmark's workload and launch configuration (200,000 anchored
    pairs, band 100, default options); 48 sampled pairs against the oracle."""
    import torch
    from paper_2301_09310_amd import salo
    _say("anchored_long full size, band 100")
    b = I.anchored_long(0, 200_000)
    q, qo, t, to = salo.to_device(b)
    out = salo.align_banded(q, qo, t, to, 100)
    torch.cuda.synchronize()
    got = tuple(x.cpu().numpy().astype(np.int64) for x in out)
    idx = np.random.default_rng(5).choice(b.n_pairs, 48, replace=False)
    sub = b.subset(idx)
    want = O.align_banded(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, 100)
    for g, w in zip(got, want):
        assert np.array_equal(g[idx], w)
    # every score is bounded by the unbanded score
    ref = salo.align_batch(q, qo, t, to)
    torch.cuda.synchronize()
    assert np.all(got[0] <= ref[0].cpu().numpy())


def test_band_validation(dev):
    from paper_2301_09310_amd import salo
    b = I.plain_small(0, 10)
    q, qo, t, to = salo.to_device(b)
    with pytest.raises(salo.SaloError):
        salo.align_banded(q, qo, t, to, -1)
    with pytest.raises(salo.SaloError):
        salo.align_banded(q, qo, t, to, 5, mode="plain")


def test_anchored_long_every_pair_digest(dev):
    """EVERY pair of the benchmark's banded workload (200,000 anchored pairs,
    band 100, default options) against the band oracle's answers, stored as
    digests in tests/golden/band_digests.json by
    tests/golden/make_band_digests.py (oracle and seeded generator only).  On
    a mismatch the chunk digests name the first 65,536-pair chunk that
    differs, and the oracle runs on its first 500 pairs to report the first
    differing pair."""
    import hashlib
    import json
    import os
    import torch
    from paper_2301_09310_amd import salo
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "band_digests.json")) as f:
        want = json.load(f)["anchored_long_band100"]
    b = I.anchored_long(0, want["pairs"])
    assert b.sha256() == want["dataset_sha256"], "the generator changed; rerun the script"
    _say("anchored_long every pair, band", want["band"])
    q, qo, t, to = salo.to_device(b)
    out = salo.align_banded(q, qo, t, to, want["band"])
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    got = tuple(x.cpu().numpy() for x in out)
    del q, qo, t, to, out
    torch.cuda.empty_cache()
    dig = lambda a: hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()
    if all(dig(g) == want[k] for g, k in zip(got, ("score", "q_end", "t_end"))):
        return
    chunk = want["chunk_pairs"]
    for c, wd in enumerate(want["chunks"]):
        h = hashlib.sha256()
        for a in got:
            h.update(np.ascontiguousarray(a[c * chunk:(c + 1) * chunk], dtype="<i4").tobytes())
        if h.hexdigest() != wd:
            break
    idx = np.arange(c * chunk, min(b.n_pairs, c * chunk + 500))
    sub = b.subset(idx)
    w = O.align_banded(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, want["band"])
    for k, p in enumerate(idx):
        g3, w3 = tuple(int(x[p]) for x in got), tuple(int(x[k]) for x in w)
        assert g3 == w3, "pair %d: gpu %s, oracle %s" % (p, g3, w3)
    raise AssertionError("chunk %d differs, but not in its first %d pairs" % (c, len(idx)))
