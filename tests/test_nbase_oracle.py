"""Pins of the oracles' N rule (CPU only).

Reads carry a fifth letter, N, for an unknown base (SALoBa, Section II-B).
Reading taken: an N scores the mismatch against every base, N included.
The 2-bit stream keeps A/C/G/T codes and an N mask (bit k of word k>>5)
marks N bases.  Pins:
  * exhaustive path enumeration on tiny strings over ACGTN (the brute-force
    substitution score treats N as never matching) for score and end, and
    for start positions;
  * closed forms: an all-N query scores 0; an empty mask changes nothing;
  * packing: N/n become mask bits (and bases), other letters stay invalid;
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
ROOT = os.path.dirname(HERE)
SCORINGS = [(1, -4, 6, 1), (2, -3, 1, 2), (1, -1, 0, 1), (3, -4, 2, 0)]


def batch_n(qs, ts):
    """Packed batch and N masks of strings over ACGTN."""
    b = I.from_strings([q.replace("N", "A") for q in qs], [t.replace("N", "A") for t in ts])

    def mask(strs):
        text = "".join(strs)
        m = np.zeros(max((len(text) + 31) // 32, 1), np.uint32)
        for k, c in enumerate(text):
            if c == "N":
                m[k >> 5] |= np.uint32(1 << (k & 31))
        return m
    return b, mask(qs), mask(ts)


def _tiny(seed, count):
    rng = random.Random(seed)
    return [("".join(rng.choice("ACGN") for _ in range(rng.randint(1, 5))),
             "".join(rng.choice("ACGN") for _ in range(rng.randint(1, 5)))) for _ in range(count)]


def _check_bruteforce(align, starts, seed=0, count=30):
    for sc in SCORINGS:
        cases = _tiny(seed + 5 * sc[0] + sc[2], count)
        b, qm, tm = batch_n([c[0] for c in cases], [c[1] for c in cases])
        r = align(b, qm, tm, sc)
        try:
            st = starts(b, qm, tm, r, sc)
        except RuntimeError:        # answers the start recurrence cannot reach
            return False
        for k, (q, t) in enumerate(cases):
            H = B.enumerate_h(q, t, sc)
            want = B.first_max(H)
            if tuple(int(x[k]) for x in r) != want:
                return False
            if want[0] > 0:
                best, opts = B.enumerate_starts(q, t, sc, want[1], want[2])
                if best != want[0] or (int(st[1][k]), int(st[0][k])) != max(opts):
                    return False
    return True


def _oracle_align(b, qm, tm, sc):
    return O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, sc,
                         q_nmask=qm, t_nmask=tm)


def _oracle_starts(b, qm, tm, r, sc):
    return O.start_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, *r, scoring=sc,
                         q_nmask=qm, t_nmask=tm)


def test_bruteforce_with_n():
    assert _check_bruteforce(_oracle_align, _oracle_starts)


def test_first_max_convention():
    assert B.first_max([[0, 2], [2, 1]]) == (2, 1, 0)


def test_all_n_query_scores_zero():
    b, qm, tm = batch_n(["NNNNNN", "N"], ["ACGTNN", "N"])
    r = _oracle_align(b, qm, tm, (1, -4, 6, 1))
    assert r[0].tolist() == [0, 0] and r[1].tolist() == [-1, -1] and r[2].tolist() == [-1, -1]


def test_n_separates_runs():
    # ACGT N ACGT against itself: the N costs 4, so the runs score 4 each
    # and the first maximum is the end of the first run
    b, qm, tm = batch_n(["ACGTNACGT"], ["ACGTNACGT"])
    r = _oracle_align(b, qm, tm, (1, -4, 6, 1))
    assert (int(r[0][0]), int(r[1][0]), int(r[2][0])) == (4, 3, 3)


def test_empty_mask_changes_nothing():
    b = I.random_pairs(3, 200, 80)
    plain = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    zq = np.zeros((int(b.q_offsets[-1]) + 31) // 32 + 1, np.uint32)
    zt = np.zeros((int(b.t_offsets[-1]) + 31) // 32 + 1, np.uint32)
    masked = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, q_nmask=zq, t_nmask=zt)
    for x, y in zip(plain, masked):
        assert np.array_equal(x, y)


def test_pack_with_n_mask():
    text = "ACGNnTXN"
    chars = np.frombuffer(text.encode(), np.uint8)
    out, bad, mask = O.pack(chars, nmask=True)
    assert bad == 1                                   # only X is invalid
    assert int(mask[0]) == (1 << 3) | (1 << 4) | (1 << 7)
    # codes: A C G N(0) n(0) T X(0) N(0)
    assert out[:2].tobytes() == bytes([0 | 1 << 2 | 2 << 4, 3 << 2])
    # reverse complement: mirrored N stays N
    rc, bad_rc, mask_rc = O.pack(chars, np.array([0, 8], np.int64), revcomp=True, nmask=True)
    assert bad_rc == 1 and int(mask_rc[0]) == (1 << 0) | (1 << 3) | (1 << 4)
    _, bad_plain = O.pack(chars)
    assert bad_plain == 4                             # without a mask N and n are invalid


MUTANTS = {
    "gotoh_oracle.c": {
        "n_matches_n": ("const int64_t s = (t_is_n || is_n(qn, q0 + j)) ? mismatch : s_acgt;",
                        "const int64_t s = (t_is_n && is_n(qn, q0 + j)) ? mismatch : s_acgt;"),
        "target_n_ignored": ("const int64_t s = (t_is_n || is_n(qn, q0 + j)) ? mismatch : s_acgt;",
                             "const int64_t s = is_n(qn, q0 + j) ? mismatch : s_acgt;"),
        "query_n_ignored": ("const int64_t s = (t_is_n || is_n(qn, q0 + j)) ? mismatch : s_acgt;",
                            "const int64_t s = t_is_n ? mismatch : s_acgt;"),
        "mask_bit_order": ("return mask != NULL && ((mask[k >> 5] >> (k & 31)) & 1u);",
                           "return mask != NULL && ((mask[k >> 5] >> (31 - (k & 31))) & 1u);"),
    },
}


def _lib_fns(so):
    lib = ctypes.CDLL(so)
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_align_batch_n.argtypes = [p, p, p, p, p, p, i64, i64, i64, i64, i64, p, p, p,
                                         ctypes.c_int]

    def align(b, qm, tm, sc):
        n = b.n_pairs
        out = [np.zeros(n, np.int64) for _ in range(3)]
        lib.oracle_align_batch_n(b.q_seqs.ctypes.data, qm.ctypes.data, b.q_offsets.ctypes.data,
                                 b.t_seqs.ctypes.data, tm.ctypes.data, b.t_offsets.ctypes.data,
                                 n, *sc, *(o.ctypes.data for o in out), 1)
        return out
    return align


@pytest.mark.parametrize("name", sorted(MUTANTS["gotoh_oracle.c"]))
def test_planted_mistake_is_caught(name):
    src = open(os.path.join(ROOT, "oracle", "gotoh_oracle.c")).read()
    old, new = MUTANTS["gotoh_oracle.c"][name]
    assert src.count(old) == 1, "mutation site moved: %s" % name
    with tempfile.TemporaryDirectory() as tmp:
        fns = {}
        for tag, text in (("real", src), (name, src.replace(old, new))):
            c = os.path.join(tmp, tag + ".c")
            so = os.path.join(tmp, tag + ".so")
            open(c, "w").write(text)
            subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", so,
                            c], check=True)
            fns[tag] = _lib_fns(so)
        assert _check_bruteforce(fns["real"], _oracle_starts, seed=7, count=25)
        assert not _check_bruteforce(fns[name], _oracle_starts, seed=7, count=25)
