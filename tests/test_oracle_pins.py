"""Pins for the CPU oracle (Section II-A, Eq. 1), independent of the oracle
itself and of the GPU path.  CPU only.

Every check reaches its expected value by another route than Eq. 1:
exhaustive enumeration of alignments, textbook special cases, hand-derived
closed forms (tests/golden/hand_derived.txt) and invariants of local
alignment.
"""
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from tests import bruteforce as B

SCORINGS = [(1, -4, 6, 1), (2, -3, 5, 2), (1, -1, 1, 1), (3, 0, 2, 1),
            (1, -2, 0, 1), (5, -4, 3, 0), (1, -4, 0, 0)]
ALPHA = "ACGT"


def rand_seq(rng, n, alphabet=ALPHA):
    return "".join(rng.choice(alphabet) for _ in range(n))


def oracle_table(q, t, scoring):
    """Every H(i, j) of the oracle's table, one cell at a time."""
    from paper_2301_09310_amd import inputs as I
    qs = I.pack_bases(I.encode(q)) if q else np.zeros(4, np.uint8)
    ts = I.pack_bases(I.encode(t)) if t else np.zeros(4, np.uint8)
    return [[O.cell_h(qs, 0, len(q), ts, 0, len(t), scoring, i, j)
             for j in range(len(q))] for i in range(len(t))]


# ------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(12))
def test_full_table_matches_exhaustive_enumeration(seed):
    """Every cell of the oracle's table equals the best enumerated path."""
    rng = random.Random(seed)
    for _ in range(6):
        m, n = rng.randint(1, 4), rng.randint(1, 4)
        # small alphabets make ties and repeats likely
        alph = ALPHA[: rng.choice([2, 3, 4])]
        q, t = rand_seq(rng, m, alph), rand_seq(rng, n, alph)
        sc = rng.choice(SCORINGS)
        want = B.enumerate_h(q, t, sc)
        got = oracle_table(q, t, sc)
        assert got == want, (q, t, sc)
        assert O.align_strings(q, t, sc) == B.first_max(want), (q, t, sc)


@pytest.mark.parametrize("seed", range(6))
def test_answer_matches_enumeration_length5(seed):
    rng = random.Random(100 + seed)
    for _ in range(3):
        m, n = rng.randint(3, 5), rng.randint(3, 5)
        q, t = rand_seq(rng, m, "AC"), rand_seq(rng, n, "ACG")
        sc = rng.choice(SCORINGS)
        assert O.align_strings(q, t, sc) == B.first_max(B.enumerate_h(q, t, sc))


# -------------------------------------------------------- golden fixtures

def _golden_rows():
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_derived.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = line.split()
        rows.append((f[0], f[1], tuple(int(x) for x in f[2:6]),
                     tuple(int(x) for x in f[6:9])))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: r[0][:12])
def test_hand_derived_closed_forms(row):
    q, t, sc, want = row
    assert O.align_strings(q, t, sc) == want


def test_gap_cost_reading_discriminates():
    """Eq. 1 names alpha (new gap) and beta (continued gap); the reading
    taken is that a k-base gap costs gap_open + k*gap_extend (alpha =
    o + e).  Enumeration under that cost model and under the other one
    (alpha = o) disagree on this pair, and the oracle follows the first."""
    q, t, sc = "AAACCC", "AAAGGCCC", (1, -4, 1, 1)
    ours = B.first_max(B.enumerate_h(q, t, sc))
    other = B.first_max(B.enumerate_h(q, t, (1, -4, 0, 1)))   # o+(k-1)e == 0+k*e
    assert ours == (3, 2, 2) and other == (4, 5, 7)
    assert O.align_strings(q, t, sc) == ours


# ---------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 7, 64, 300])
def test_identical_strings(n):
    rng = random.Random(n)
    s = rand_seq(rng, n)
    for a, b, o, e in SCORINGS:
        assert O.align_strings(s, s, (a, b, o, e)) == (n * a, n - 1, n - 1)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 9), (40, 17)])
def test_disjoint_alphabets_score_zero(m, n):
    for sc in SCORINGS:
        if sc[1] > 0:
            continue
        assert O.align_strings("A" * m, "C" * n, sc) == (0, -1, -1)
        assert O.align_strings("AG" * m, "CT" * n, sc) == (0, -1, -1)


def _gap_route_dominates(k, sc):
    """Crossing the G^k block with j mismatched G's and a (k-j)-base gap
    changes the score by j*(b - a + e) (plus o when j = k) relative to one
    k-base gap; the closed form below needs the pure gap to win strictly."""
    a, b, o, e = sc
    return (b - a + e) < 0 and k * (b - a + e) + o < 0


def _gap_closed_form(x, y, k, sc):
    """q = A^x C^y, t = A^x G^k C^y, when the pure gap route dominates: the
    best is both blocks bridged by one k-base deletion, or the larger block
    alone (the A block ends first in row-major order on a tie)."""
    a, b, o, e = sc
    bridged = (x + y) * a - (o + k * e)
    best_block = max(x, y) * a
    if bridged > best_block:
        return bridged, x + y - 1, x + k + y - 1
    if x >= y:
        return x * a, x - 1, x - 1
    return y * a, x + y - 1, x + k + y - 1


def test_gap_closed_form_agrees_with_enumeration_small():
    checked = 0
    for x in range(1, 4):
        for y in range(1, 4):
            for k in range(1, 3):
                for sc in [(1, -4, 1, 1), (2, -3, 1, 0), (3, -5, 2, 1),
                           (1, -4, 6, 1), (1, -4, 3, 1)]:
                    if not _gap_route_dominates(k, sc):
                        continue
                    q, t = "A" * x + "C" * y, "A" * x + "G" * k + "C" * y
                    want = B.first_max(B.enumerate_h(q, t, sc))
                    assert _gap_closed_form(x, y, k, sc) == want, (x, y, k, sc)
                    checked += 1
    assert checked > 40


def test_mismatch_route_beats_single_base_gap():
    """With (1,-4,6,1) and k = 1 the G is cheaper as a mismatch (-4 and one
    lost match) than as a gap (-7): 9 + 39 - 4 = 44, ending on the diagonal."""
    q, t = "A" * 9 + "C" * 40, "A" * 9 + "G" + "C" * 40
    assert O.align_strings(q, t, (1, -4, 6, 1)) == (44, 48, 48)


@pytest.mark.parametrize("x,y,k", [(12, 12, 3), (30, 7, 5), (9, 40, 2), (50, 50, 20)])
def test_gap_closed_form_large(x, y, k):
    for sc in [(1, -4, 6, 1), (2, -3, 5, 2), (1, -4, 1, 1), (3, -1, 4, 0)]:
        if not _gap_route_dominates(k, sc):
            continue
        q, t = "A" * x + "C" * y, "A" * x + "G" * k + "C" * y
        assert O.align_strings(q, t, sc) == _gap_closed_form(x, y, k, sc)
        # mirrored: the G block in the query is a gap along the query (E of
        # Eq. 1); ends swap with the roles of the strings
        s, qe, te = _gap_closed_form(x, y, k, sc)
        got = O.align_strings(t, q, sc)
        if s > max(x, y) * sc[0]:
            assert got == (s, te, qe)
        else:
            assert got[0] == s


# ---------------------------------------------------- textbook reductions

@pytest.mark.parametrize("seed", range(8))
def test_ungapped_case_is_kadane_on_diagonals(seed):
    """gap_open >= match*min(m,n) makes every gapped path score <= 0."""
    rng = random.Random(1000 + seed)
    m, n = rng.randint(1, 30), rng.randint(1, 30)
    q, t = rand_seq(rng, m, "ACG"), rand_seq(rng, n, "ACG")
    a = rng.randint(1, 3)
    sc = (a, -rng.randint(0, 4), a * min(m, n), rng.randint(0, 2))
    want = B.kadane_table(q, t, sc)
    assert O.align_strings(q, t, sc) == B.first_max(want)
    if m * n <= 120:
        assert oracle_table(q, t, sc) == want


@pytest.mark.parametrize("seed", range(8))
def test_zero_gap_open_is_linear_gap_smith_waterman(seed):
    rng = random.Random(2000 + seed)
    m, n = rng.randint(1, 40), rng.randint(1, 40)
    q, t = rand_seq(rng, m), rand_seq(rng, n)
    a, b, e = rng.randint(1, 3), -rng.randint(0, 4), rng.randint(0, 3)
    want = B.linear_sw_table(q, t, a, b, e)
    assert O.align_strings(q, t, (a, b, 0, e)) == B.first_max(want)
    if m * n <= 150:
        assert oracle_table(q, t, (a, b, 0, e)) == want


@pytest.mark.parametrize("seed", range(8))
def test_prohibitive_penalties_give_longest_common_substring(seed):
    rng = random.Random(3000 + seed)
    m, n = rng.randint(1, 40), rng.randint(1, 40)
    q, t = rand_seq(rng, m, "AC"), rand_seq(rng, n, "ACG")
    a = rng.randint(1, 3)
    big = a * min(m, n)
    L = B.common_suffix_table(q, t)
    want = B.first_max([[a * v for v in row] for row in L])
    assert O.align_strings(q, t, (a, -big, big, 1)) == want


# ------------------------------------------------------------- invariants

def _complement(s):
    return s.translate(str.maketrans("ACGT", "TGCA"))


@pytest.mark.parametrize("seed", range(10))
def test_invariants(seed):
    rng = random.Random(4000 + seed)
    m, n = rng.randint(0, 60), rng.randint(0, 60)
    q, t = rand_seq(rng, m), rand_seq(rng, n)
    if m and n and rng.random() < 0.5:   # make some pairs related
        k = rng.randint(0, n - 1)
        q = (t[k:k + m] + q)[:m]
    sc = rng.choice(SCORINGS)
    a, b, o, e = sc
    s, qe, te = O.align_strings(q, t, sc)
    assert 0 <= s <= a * min(m, n)
    assert (s == 0) == (qe == -1) == (te == -1)
    # reversing both strings keeps the score
    assert O.align_strings(q[::-1], t[::-1], sc)[0] == s
    # swapping query and target keeps the score
    assert O.align_strings(t, q, sc)[0] == s
    # one alphabet permutation on both keeps score and ends
    assert O.align_strings(_complement(q), _complement(t), sc) == (s, qe, te)
    # harsher penalties never raise the score
    assert O.align_strings(q, t, (a, b, o + 1, e))[0] <= s
    assert O.align_strings(q, t, (a, b, o, e + 1))[0] <= s
    assert O.align_strings(q, t, (a, b - 1, o, e))[0] <= s
    # appending bases never lowers the score
    assert O.align_strings(q + "A", t, sc)[0] >= s
    assert O.align_strings(q, "G" + t, sc)[0] >= s
    # the reported end holds the score
    if s:
        from paper_2301_09310_amd import inputs as I
        qs, ts = I.pack_bases(I.encode(q)), I.pack_bases(I.encode(t))
        assert O.cell_h(qs, 0, m, ts, 0, n, sc, te, qe) == s


def test_clamping_e_and_f_at_zero_leaves_h_unchanged():
    """Boundary values of E/F at or below 0 (and clamping E, F at 0) give
    the same H everywhere -- the property the GPU's saturating 16-bit
    arithmetic relies on.  Checked against the oracle's table."""
    rng = random.Random(5)
    for _ in range(40):
        m, n = rng.randint(1, 12), rng.randint(1, 12)
        q, t = rand_seq(rng, m), rand_seq(rng, n)
        sc = rng.choice(SCORINGS)
        a, b, o, e = sc
        al, be = o + e, e
        H = [[0] * m for _ in range(n)]
        F = [0] * m
        for i in range(n):
            E = 0
            for j in range(m):
                hl = H[i][j - 1] if j else 0
                hu = H[i - 1][j] if i else 0
                hd = H[i - 1][j - 1] if i and j else 0
                E = max(0, hl - al, E - be)
                F[j] = max(0, hu - al, F[j] - be)
                H[i][j] = max(0, E, F[j], hd + (a if t[i] == q[j] else b))
        assert oracle_table(q, t, sc) == H


# --------------------------------------------------------- batch plumbing

def test_batch_threads_and_order_do_not_matter():
    from paper_2301_09310_amd import inputs as I
    b = I.random_pairs(7, 300, 90)
    r1 = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, nthreads=1)
    r8 = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, nthreads=8)
    for x, y in zip(r1, r8):
        assert np.array_equal(x, y)
    # each pair alone gives the same answer as in the batch
    for p in range(0, 300, 37):
        q, t = b.pair_strings(p)
        assert O.align_strings(q, t) == (r1[0][p], r1[1][p], r1[2][p])


def test_empty_pairs():
    from paper_2301_09310_amd import inputs as I
    b = I.from_strings(["", "ACGT", "", "A"], ["ACGT", "", "", "A"])
    s, qe, te = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    assert s.tolist() == [0, 0, 0, 1]
    assert qe.tolist() == [-1, -1, -1, 0]
    assert te.tolist() == [-1, -1, -1, 0]
