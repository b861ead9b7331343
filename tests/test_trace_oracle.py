"""Pins of the trace oracle (CPU only).

The trace of a pair is one optimal alignment from its start to its end
(Section II-A: the path that reaches the highest cell), chosen by a fixed
order of preference while walking back from the end.  Pins:
  * exhaustive enumeration of every alignment path between start and end
    on tiny strings (gap runs split into several gaps included): the best
    enumerated score is the pair's score, and the oracle's CIGAR is that of
    the optimal path whose sequence of backward choices is smallest;
  * hand-derived traces (tests/golden/trace_examples.txt);
  * on larger random pairs: the CIGAR covers exactly q[q_start..q_end] and
    t[t_start..t_end], '=' and 'X' agree with the bases, its score
    recomputed from the runs is the pair's score, and it begins and ends
    with equal bases;
and planted mistakes in copies of the oracle must fail these pins.
"""
import ctypes
import os
import random
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "trace_oracle.c")
GOLDEN = os.path.join(HERE, "golden", "trace_examples.txt")
SCORINGS = [(1, -4, 6, 1), (2, -3, 2, 1), (1, -1, 0, 1), (2, -1, 1, 1), (3, -2, 0, 2)]
CODE = {"=": 7, "X": 8, "I": 1, "D": 2}


def answers(b, sc):
    s, qe, te = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, sc)
    qs, ts = O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, s, qe, te, scoring=sc)
    return s, qs, qe, ts, te


def best_trace(q, t, sc, qs, qe, ts, te):
    """Every state path from the pair (ts, qs) to (te, qe) by exhaustive
    search: ops '=', 'X', and gaps 'I' / 'D' that either open (alpha) or,
    right after the same kind of gap, extend (beta).  Returns the best
    score and the CIGAR of the optimal path whose backward choice sequence
    is smallest: in state H pair < I < D, in a gap state open < extend."""
    a, b, o, e = sc
    alpha, beta = o + e, e
    sys.setrecursionlimit(10000)
    paths = []

    def walk(i, j, ops, score):
        # (i, j): last consumed target / query index
        if i == te and j == qe:
            paths.append((score, list(ops)))
        if i + 1 <= te and j + 1 <= qe:
            eq = t[i + 1] == q[j + 1]
            ops.append(("=" if eq else "X", 0))
            walk(i + 1, j + 1, ops, score + (a if eq else b))
            ops.pop()
        if j + 1 <= qe:
            for ext in (0, 1):
                if ext and (not ops or ops[-1][0] != "I"):
                    continue
                ops.append(("I", ext))
                walk(i, j + 1, ops, score - (beta if ext else alpha))
                ops.pop()
        if i + 1 <= te:
            for ext in (0, 1):
                if ext and (not ops or ops[-1][0] != "D"):
                    continue
                ops.append(("D", ext))
                walk(i + 1, j, ops, score - (beta if ext else alpha))
                ops.pop()

    eq = t[ts] == q[qs]
    walk(ts, qs, [("=" if eq else "X", 0)], a if eq else b)
    best = max(p[0] for p in paths)

    def choices(ops):
        out, state = [], "H"
        for op, ext in reversed(ops):
            if state == "H":
                if op in "=X":
                    out.append(0)
                    continue
                out.append(1 if op == "I" else 2)
                state = op
            out.append(1 if ext else 0)
            state = op if ext else "H"
        return out
    chosen = min((p for p in paths if p[0] == best), key=lambda p: choices(p[1]))[1]
    runs = []
    for op, _ in chosen:
        if runs and runs[-1][1] == op:
            runs[-1][0] += 1
        else:
            runs.append([1, op])
    return best, "".join("%d%s" % (n, op) for n, op in runs)


def _tiny_cases(seed, count, max_len=6):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        alph = "ACGT"[: rng.choice([2, 3, 4])]
        out.append(("".join(rng.choice(alph) for _ in range(rng.randint(1, max_len))),
                    "".join(rng.choice(alph) for _ in range(rng.randint(1, max_len)))))
    return out


def _check_bruteforce(trace_fn, seed=0, count=40):
    for sc in SCORINGS:
        cases = _tiny_cases(seed + sc[0] * 7 + sc[2], count)
        b = I.from_strings([c[0] for c in cases], [c[1] for c in cases])
        s, qs, qe, ts, te = answers(b, sc)
        try:
            off, cig, ln = trace_fn(b, s, qs, qe, ts, te, sc)
        except RuntimeError:
            return False
        for k, (q, t) in enumerate(cases):
            if s[k] <= 0:
                if ln[k] != 0:
                    return False
                continue
            best, want = best_trace(q, t, sc, int(qs[k]), int(qe[k]), int(ts[k]), int(te[k]))
            if best != s[k] or ln[k] < 0 or O.cigar_string(cig, off[k], ln[k]) != want:
                return False
    return True


def _oracle(b, s, qs, qe, ts, te, sc):
    return O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, s, qs, qe, ts, te, sc)


def test_bruteforce_optimal_and_preferred():
    assert _check_bruteforce(_oracle)


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        left, right = line.split("|")
        q, t, *sc = left.split()
        vals = right.split()
        rows.append((q, t, tuple(int(x) for x in sc), tuple(int(x) for x in vals[:5]), vals[5]))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: r[0] + "/" + r[1])
def test_golden(row):
    q, t, sc, want, cigar = row
    b = I.from_strings([q], [t])
    s, qs, qe, ts, te = answers(b, sc)
    assert (int(s[0]), int(qs[0]), int(qe[0]), int(ts[0]), int(te[0])) == want
    off, cig, ln = _oracle(b, s, qs, qe, ts, te, sc)
    assert O.cigar_string(cig, off[0], ln[0]) == cigar
    assert best_trace(q, t, sc, want[1], want[2], want[3], want[4]) == (want[0], cigar)


def check_consistency(b, sc, off, cig, ln, s, qs, qe, ts, te):
    a, mis, o, e = sc
    for p in range(b.n_pairs):
        if s[p] <= 0:
            assert ln[p] == 0
            continue
        q, t = b.pair_strings(p)
        runs = [(int(c) >> 4, O.CIGAR_OPS[int(c) & 15]) for c in cig[off[p]:off[p] + ln[p]]]
        assert runs and runs[0][1] == "=" and runs[-1][1] == "="
        i, j, score = int(ts[p]), int(qs[p]), 0
        for n, op in runs:
            assert n >= 1
            if op in "=X":
                for _ in range(n):
                    assert (t[i] == q[j]) == (op == "=")
                    score += a if op == "=" else mis
                    i += 1
                    j += 1
            else:
                score -= o + n * e
                if op == "I":
                    j += n
                else:
                    i += n
        assert (i, j) == (int(te[p]) + 1, int(qe[p]) + 1)
        assert score == s[p]


@pytest.mark.parametrize("sc", SCORINGS)
def test_consistent_on_random_pairs(sc):
    b = I.random_pairs(31, 120, 160, min_len=0, related=0.8)
    s, qs, qe, ts, te = answers(b, sc)
    off, cig, ln = _oracle(b, s, qs, qe, ts, te, sc)
    check_consistency(b, sc, off, cig, ln, s, qs, qe, ts, te)


def test_wrong_score_is_reported():
    b = I.from_strings(["ACGTACGT"], ["ACGTTACGT"])
    s, qs, qe, ts, te = answers(b, (2, -3, 2, 1))
    with pytest.raises(RuntimeError):
        _oracle(b, s + 1, qs, qe, ts, te, (2, -3, 2, 1))


MUTANTS = {
    "f_before_e": ("} else if (AT(H, i, j) == AT(E, i, j)) {",
                   "} else if (AT(H, i, j) != AT(F, i, j)) {"),
    "extend_first_in_e": ("if (AT(E, i, j) == AT(H, i, j - 1) - alpha) state = 0;",
                          "if (AT(E, i, j) != AT(E, i, j - 1) - beta) state = 0;"),
    "extend_first_in_f": ("if (AT(F, i, j) == AT(H, i - 1, j) - alpha) state = 0;",
                          "if (AT(F, i, j) != AT(F, i - 1, j) - beta) state = 0;"),
    "i_d_swapped": ("#define OP_I 1\n#define OP_D 2", "#define OP_I 2\n#define OP_D 1"),
    "eq_x_swapped": ("op = ti == qj ? OP_EQ : OP_X;", "op = ti == qj ? OP_X : OP_EQ;"),
    "runs_not_reversed": ("cig[cig_off[p] + k] = rev[nrev - 1 - k];",
                          "cig[cig_off[p] + k] = rev[k];"),
    "beta_for_open": ("AT(E, i, j) = max2(max2(AT(H, i, j - 1) - alpha,",
                      "AT(E, i, j) = max2(max2(AT(H, i, j - 1) - beta,"),
}


def _mutant(text, tmp, name):
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    open(c, "w").write(text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", so, c], check=True)
    lib = ctypes.CDLL(so)
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_trace_batch.argtypes = [p, p, p, p, i64, i64, i64, i64, i64,
                                       p, p, p, p, p, p, p, p]
    lib.oracle_trace_batch.restype = i64

    def fn(b, s, qs, qe, ts, te, sc):
        off = O.cigar_capacity(b.q_offsets, b.t_offsets)
        cig = np.zeros(max(int(off[-1]), 1), np.uint32)
        ln = np.zeros(b.n_pairs, np.int64)
        arr = [np.ascontiguousarray(x, dtype=np.int64) for x in (s, qs, qe, ts, te)]
        bad = lib.oracle_trace_batch(b.q_seqs.ctypes.data, b.q_offsets.ctypes.data,
                                     b.t_seqs.ctypes.data, b.t_offsets.ctypes.data,
                                     b.n_pairs, *sc, *(x.ctypes.data for x in arr),
                                     off.ctypes.data, cig.ctypes.data, ln.ctypes.data)
        if bad != 0:
            raise RuntimeError("inconsistent")
        return off, cig, ln
    return fn


def _passes_all(fn):
    if not _check_bruteforce(fn, seed=5, count=25):
        return False
    for q, t, sc, want, cigar in _golden():
        b = I.from_strings([q], [t])
        s, qs, qe, ts, te = answers(b, sc)
        try:
            off, cig, ln = fn(b, s, qs, qe, ts, te, sc)
        except RuntimeError:
            return False
        if O.cigar_string(cig, off[0], ln[0]) != cigar:
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved: %s" % name
    with tempfile.TemporaryDirectory() as tmp:
        assert _passes_all(_mutant(src, tmp, "real"))
        assert not _passes_all(_mutant(src.replace(old, new), tmp, name))


def test_threaded_calls_agree():
    b = I.random_pairs(33, 90, 150, related=0.8)
    s, qs, qe, ts, te = answers(b, (1, -4, 6, 1))
    one = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, s, qs, qe, ts, te)
    many = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, s, qs, qe, ts, te,
                         threads=6)
    for x, y in zip(one, many):
        assert np.array_equal(x, y)
