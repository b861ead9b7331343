"""Planted-mistake check for the oracle's pins (CPU only).

Each mutant is a copy of oracle/gotoh_oracle.c with one plausible mistake
(a dropped term, a wrong sign, a swapped operand, an off-by-one, a changed
tie rule).  The mutant is compiled to a temporary library and run through
a quick subset of the independent pins; every mutant must fail at least
one of them.  The real oracle must pass the same subset.
"""
import ctypes
import os
import random
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2301_09310_amd import inputs as I
from tests import bruteforce as B

SRC = os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle",
                   "gotoh_oracle.c")

MUTANTS = {
    "alpha_is_open_only": ("jb.alpha = gap_open + gap_extend;", "jb.alpha = gap_open;"),
    "beta_is_open": ("jb.beta = gap_extend;", "jb.beta = gap_open;"),
    "no_zero_floor": ("if (h < 0) h = 0;\n            h_diag = Hrow[j];   /* becomes",
                      "h_diag = Hrow[j];   /* becomes"),
    "e_ignores_extension": ("e = e_open > e_ext ? e_open : e_ext;", "e = e_open;"),
    "f_ignores_extension": ("const int64_t f = f_open > f_ext ? f_open : f_ext;",
                            "const int64_t f = f_open;"),
    "f_not_stored": ("Frow[j] = f;\n            h_left = h;\n            if (h > best) {     /*",
                     "h_left = h;\n            if (h > best) {     /*"),
    "diag_not_shifted": ("h_diag = Hrow[j];   /* becomes", "h_diag = h_diag;   /* becomes"),
    "last_max_not_first": ("if (h > best) {     /* strict", "if (h >= best && h > 0) {     /* strict"),
    "ends_swapped": ("*qend = best > 0 ? bj : -1;\n    *tend = best > 0 ? bi : -1;",
                     "*qend = best > 0 ? bi : -1;\n    *tend = best > 0 ? bj : -1;"),
    "mismatch_as_match": ("(ti == qj) ? match : mismatch", "(ti != qj) ? match : mismatch"),
    "base_bits_msb_first": ("return (packed[k >> 2] >> (2 * (k & 3))) & 3;",
                            "return (packed[k >> 2] >> (6 - 2 * (k & 3))) & 3;"),
    "e_from_up_cell": ("const int64_t e_open = h_left - alpha;",
                       "const int64_t e_open = Hrow[j] - alpha;"),
}


def _build(src_text, tmpdir, name):
    c = os.path.join(tmpdir, name + ".c")
    so = os.path.join(tmpdir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread",
                    "-o", so, c], check=True)
    lib = ctypes.CDLL(so)
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_align_batch.argtypes = [p, p, p, p, i64, i64, i64, i64, i64,
                                       p, p, p, ctypes.c_int]
    return lib


def _align(lib, b, sc):
    n = b.n_pairs
    out = [np.zeros(n, np.int64) for _ in range(3)]
    a, mm, o, e = sc
    lib.oracle_align_batch(b.q_seqs.ctypes.data, b.q_offsets.ctypes.data,
                           b.t_seqs.ctypes.data, b.t_offsets.ctypes.data, n,
                           a, mm, o, e, out[0].ctypes.data, out[1].ctypes.data,
                           out[2].ctypes.data, 1)
    return list(zip(*(x.tolist() for x in out)))


def _cases():
    """(batch, scoring, expected answers) from the independent routes."""
    rng = random.Random(77)
    cases = []
    scorings = [(1, -4, 6, 1), (2, -3, 1, 2), (1, -1, 0, 1), (3, -4, 2, 0)]
    for sc in scorings:
        qs, ts = [], []
        for _ in range(25):
            m, n = rng.randint(1, 4), rng.randint(1, 4)
            alph = "ACGT"[: rng.choice([2, 4])]
            qs.append("".join(rng.choice(alph) for _ in range(m)))
            ts.append("".join(rng.choice(alph) for _ in range(n)))
        want = [B.first_max(B.enumerate_h(q, t, sc)) for q, t in zip(qs, ts)]
        cases.append((I.from_strings(qs, ts), sc, want))
    # longer pairs: linear-gap textbook SW and the gap closed form
    qs, ts = [], []
    for _ in range(10):
        m, n = rng.randint(10, 40), rng.randint(10, 40)
        qs.append("".join(rng.choice("ACGT") for _ in range(m)))
        ts.append("".join(rng.choice("ACGT") for _ in range(n)))
    want = [B.first_max(B.linear_sw_table(q, t, 2, -3, 1)) for q, t in zip(qs, ts)]
    cases.append((I.from_strings(qs, ts), (2, -3, 0, 1), want))
    q, t = "A" * 12 + "C" * 12, "A" * 12 + "GGG" + "C" * 12
    # the same gap on either side: a deletion from the target (F direction)
    # and an insertion in the query (E direction)
    cases.append((I.from_strings([q, q, t], [t, q, q]), (1, -4, 6, 1),
                  [(15, 23, 26), (24, 23, 23), (15, 26, 23)]))
    return cases


@pytest.fixture(scope="module")
def built():
    tmp = tempfile.mkdtemp(prefix="oracle_mutants_")
    text = open(SRC).read()
    libs = {"original": _build(text, tmp, "original")}
    for name, (old, new) in MUTANTS.items():
        assert text.count(old) == 1, name
        libs[name] = _build(text.replace(old, new), tmp, name)
    return libs


def test_original_passes_quick_pins(built):
    for b, sc, want in _cases():
        assert _align(built["original"], b, sc) == want


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_is_caught(built, name):
    caught = any(_align(built[name], b, sc) != want for b, sc, want in _cases())
    assert caught, "mutant %s survived the pins" % name
