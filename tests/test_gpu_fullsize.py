"""Every pair of the four batch workloads on the GPU, in the benchmark's
launch configuration (salo_align_batch with default options: persistent,
length-binned), compared with the oracle's answers for every pair.

The oracle's answers for the whole batches are stored as sha256 digests in
tests/golden/full_digests.json, written by tests/golden/make_full_digests.py,
which runs only the CPU oracle and the seeded generator (about an hour of
CPU for the 4M-pair mixed batch, so they are computed once, not per run).
A test first checks that the generator still produces the batch the digests
were taken on (dataset sha256), then compares the digest of each GPU output
array (int32, little-endian) with the oracle's.  On a mismatch the
per-65,536-pair chunk digests name the chunks that differ, and the oracle is
run on the first of them to report the first differing pair.  Range
properties that hold for every pair are checked too.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu
SCORING = (1, -4, 6, 1)
HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "full_digests.json")


def _table():
    with open(DIGESTS) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_09310_amd import salo
    salo.load()
    return torch.device("cuda:0")


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def _chunk_digests(got, chunk):
    out = []
    for c0 in range(0, len(got[0]), chunk):
        h = hashlib.sha256()
        for a in got:
            h.update(np.ascontiguousarray(a[c0:c0 + chunk], dtype="<i4").tobytes())
        out.append(h.hexdigest())
    return out


def _run_full(b):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = salo.to_device(b)
    out = salo.align_batch(q, qo, t, to, SCORING)     # salo_align_batch itself
    torch.cuda.synchronize()
    assert salo.error_count() == 0
    res = tuple(x.cpu().numpy() for x in out)
    del q, qo, t, to, out
    torch.cuda.empty_cache()
    return res


def _ranges(b, got):
    s, qe, te = (x.astype(np.int64) for x in got)
    m, n = b.q_lens(), b.t_lens()
    assert np.all(s >= 0) and np.all(s <= SCORING[0] * np.minimum(m, n))
    zero = s == 0
    assert np.all(qe[zero] == -1) and np.all(te[zero] == -1)
    assert np.all((qe[~zero] >= 0) & (qe[~zero] < m[~zero]))
    assert np.all((te[~zero] >= 0) & (te[~zero] < n[~zero]))


def _localise(b, got, rec):
    """First pair of the first differing chunk where GPU and oracle differ."""
    chunk = rec["chunk_pairs"]
    mine = _chunk_digests(got, chunk)
    bad = [k for k, (x, y) in enumerate(zip(mine, rec["chunks"])) if x != y]
    assert bad, "whole-array digests differ but no chunk does"
    c0 = bad[0] * chunk
    idx = np.arange(c0, min(b.n_pairs, c0 + chunk))
    sub = b.subset(idx)
    want = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING)
    for k, name in enumerate(("score", "q_end", "t_end")):
        diff = np.nonzero(got[k][idx].astype(np.int64) != want[k])[0]
        if diff.size:
            p = int(idx[diff[0]])
            return ("%d of %d chunks differ (first %s); %s differs at pair %d: gpu %s oracle %s"
                    % (len(bad), len(mine), bad[:8], name, p,
                       [int(x[p]) for x in got], [int(x[diff[0]]) for x in want]))
    return "chunk %d digest differs but the oracle agrees pair by pair" % bad[0]


def _full_case(name, dev):
    table = _table()
    if name not in table:
        pytest.fail("no oracle digest for %s in %s" % (name, DIGESTS))
    rec = table[name]
    b = I.WORKLOADS[name](0)
    print("[case] %s full batch, %d pairs, %.3e cells" % (name, b.n_pairs, b.cells()),
          flush=True)
    assert b.n_pairs == rec["pairs"]
    assert b.sha256() == rec["dataset_sha256"], "the generator no longer makes this batch"
    got = _run_full(b)
    _ranges(b, got)
    ok = all(_digest(got[k]) == rec[key] for k, key in enumerate(("score", "q_end", "t_end")))
    if not ok:
        pytest.fail(_localise(b, got, rec))
    sums = rec["checksums"]
    assert int(got[0].astype(np.int64).sum()) == sums["score"]
    assert int((got[0] == 0).sum()) == sums["zero_scores"]


def test_plain_small_every_pair(dev):
    _full_case("plain_small", dev)


def test_short_reads_every_pair(dev):
    _full_case("short_reads", dev)


def test_long_uneven_every_pair(dev):
    _full_case("long_uneven", dev)


@pytest.mark.timeout(600)
def test_mixed_every_pair(dev):
    _full_case("mixed", dev)
