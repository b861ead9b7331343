"""Pins of the banded oracle (CPU only).

Banded seed extension (SALoBa, Section VII-B) fills only the cells with
|i - j| <= w.  The oracle is Eq. 1 on those cells, cells outside the band
acting as the table's boundary.  Pins:
  * exhaustive enumeration of every path that stays inside the band (tiny
    strings, several widths and scorings);
  * w = 0 is the ungapped main diagonal: Kadane's running maximum along it;
  * a band at least max(m, n) wide is the unbanded oracle;
  * the score never decreases as the band widens;
and planted mistakes in copies of the oracle must fail these pins.
"""
import ctypes
import os
import random
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I
from tests import bruteforce as B

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "band_oracle.c")
SCORINGS = [(1, -4, 6, 1), (2, -3, 1, 2), (1, -1, 0, 1), (3, -4, 2, 0)]


def _cases(seed, count, max_len=5):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        alph = "ACGT"[: rng.choice([2, 4])]
        out.append(("".join(rng.choice(alph) for _ in range(rng.randint(1, max_len))),
                    "".join(rng.choice(alph) for _ in range(rng.randint(1, max_len)))))
    return out


def _check(banded, seed=0, count=30):
    for sc in SCORINGS:
        for w in (0, 1, 2, 3):
            cases = _cases(seed + 11 * w + sc[0], count)
            b = I.from_strings([c[0] for c in cases], [c[1] for c in cases])
            got = banded(b, w, sc)
            for k, (q, t) in enumerate(cases):
                want = B.first_max(B.enumerate_h(q, t, sc, band=w))
                if tuple(int(x[k]) for x in got) != want:
                    return False
    return True


def _oracle(b, w, sc):
    return O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, w, sc)


def test_bruteforce_in_band():
    assert _check(_oracle)


def test_zero_band_is_kadane_on_the_diagonal():
    b = I.random_pairs(5, 80, 40, related=0.7)
    got = _oracle(b, 0, (1, -4, 6, 1))
    for p in range(b.n_pairs):
        q, t = b.pair_strings(p)
        H = B.kadane_table(q, t, (1, -4, 6, 1))
        diag = [[H[i][j] if i == j else 0 for j in range(len(q))] for i in range(len(t))]
        assert tuple(int(x[p]) for x in got) == B.first_max(diag)


def test_wide_band_is_unbanded():
    b = I.random_pairs(6, 200, 150)
    w = 150
    got = _oracle(b, w, (2, -3, 5, 2))
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, (2, -3, 5, 2))
    for g, x in zip(got, want):
        assert np.array_equal(g, x)


def test_score_grows_with_the_band():
    b = I.random_pairs(7, 150, 200, related=0.8)
    prev = None
    for w in (0, 2, 5, 10, 30, 100, 200):
        s = _oracle(b, w, (1, -4, 6, 1))[0]
        if prev is not None:
            assert np.all(s >= prev)
        prev = s


# Resetting E and F outside the band cannot be planted as a mistake: the band
# is contiguous in every row and column, so an out-of-band cell before the
# band only ever holds the initial boundary values of E and F, and one after
# it only feeds other out-of-band cells.  Only H leaks (test_h_mask_suffices).
MUTANTS = {
    "one_sided_band": ("return d <= w && d >= -w;", "return d <= w;"),
    "band_off_by_one": ("return d <= w && d >= -w;", "return d < w && d > -w;"),
    "outside_keeps_column_h": ("                        h = 0;\n",
                               "                        h = Hrow[j];\n"),
    "outside_keeps_row_h": ("                        h = 0;\n",
                            "                        h = h_left;\n"),
}


def test_h_mask_suffices():
    """Removing the E and F resets leaves every answer unchanged."""
    src = open(SRC).read()
    mut = src.replace("                        f = BAND_NEG_INF;\n", "                        f = Frow[j];\n")
    mut = mut.replace("                        e = BAND_NEG_INF;\n", "")
    assert mut.count("BAND_NEG_INF;") < src.count("BAND_NEG_INF;")
    b = I.random_pairs(8, 60, 120, related=0.6)
    with tempfile.TemporaryDirectory() as tmp:
        fn = _mutant(mut, tmp, "hmask")
        for w in (0, 1, 4, 17, 40):
            got = fn(b, w, (1, -4, 6, 1))
            want = _oracle(b, w, (1, -4, 6, 1))
            for g, x in zip(got, want):
                assert np.array_equal(g, x)


def _mutant(text, tmp, name):
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    open(c, "w").write(text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", so, c], check=True)
    lib = ctypes.CDLL(so)
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_align_banded.argtypes = [p, p, p, p, i64, i64, i64, i64, i64, i64, p, p, p]

    def fn(b, w, sc):
        out = [np.zeros(b.n_pairs, np.int64) for _ in range(3)]
        lib.oracle_align_banded(b.q_seqs.ctypes.data, b.q_offsets.ctypes.data,
                                b.t_seqs.ctypes.data, b.t_offsets.ctypes.data, b.n_pairs,
                                *sc, w, *(x.ctypes.data for x in out))
        return out
    return fn


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved: %s" % name
    with tempfile.TemporaryDirectory() as tmp:
        assert _check(_mutant(src, tmp, "real"), seed=3, count=25)
        assert not _check(_mutant(src.replace(old, new), tmp, name), seed=3, count=25)


def test_threaded_calls_agree():
    b = I.random_pairs(9, 97, 120, related=0.7)
    one = O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, 9, threads=1)
    many = O.align_banded(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, 9, threads=7)
    for x, y in zip(one, many):
        assert np.array_equal(x, y)


def test_band_cell_count():
    rng = np.random.default_rng(4)
    ql = rng.integers(0, 40, 60)
    tl = rng.integers(0, 40, 60)
    for w in (0, 1, 5, 50):
        got = I.band_cells(ql, tl, w)
        for p in range(60):
            want = sum(1 for i in range(tl[p]) for j in range(ql[p]) if abs(i - j) <= w)
            assert got[p] == want


def test_anchored_workload_shape():
    b = I.anchored_long(0, 2000)
    ql, tl = b.q_lens(), b.t_lens()
    assert b.n_pairs == 2000
    assert ql.min() >= 250 and ql.max() <= 8000
    # the source starts the target: the best path starts at or near (0, 0)
    sub = b.subset(np.arange(20))
    s, qe, te = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets)
    qs, ts = O.start_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, s, qe, te)
    assert np.all(qs <= 64) and np.all(ts <= 64)
    # and a band of 100 keeps the whole best alignment for nearly every pair
    bs, _, _ = O.align_banded(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, 100)
    assert np.mean(bs == s) >= 0.9
