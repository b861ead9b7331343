"""Pins of the packing oracle (CPU only).

The oracle packs character reads into the aligner's 2-bit stream, forward
or reverse-complemented per sequence.  It is pinned to:
  * hand-derived examples (tests/golden/pack_examples.txt);
  * the input generator's own packer (independent code) on random reads;
  * the textbook reverse complement written with Python string operations;
  * the alignment itself: aligning the oracle-packed reads gives the same
    answers as aligning the strings;
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

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "pack_oracle.c")
RC = str.maketrans("ACGTacgt", "TGCAtgca")


def _golden():
    out = []
    for line in open(os.path.join(HERE, "golden", "pack_examples.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        chars, mode, offs, hexs, bad = [x.strip() for x in line.split("|")]
        out.append((chars, mode == "rc", np.array([int(x) for x in offs.split(",")], np.int64),
                    bytes.fromhex(hexs), int(bad)))
    return out


def _chars(s):
    return np.frombuffer(s.encode(), np.uint8)


def _reads(seed, n, max_len, alphabet="ACGT"):
    rng = random.Random(seed)
    seqs = ["".join(rng.choice(alphabet) for _ in range(rng.randint(0, max_len)))
            for _ in range(n)]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum([len(s) for s in seqs])
    return seqs, off


def _gen_pack(seqs):
    """The input generator's packer over the concatenation."""
    codes = I.encode("".join(seqs).upper()) if seqs else np.zeros(0, np.uint8)
    return I.pack_bases(codes)


@pytest.mark.parametrize("case", _golden(), ids=lambda c: "%s-%s" % (c[0], "rc" if c[1] else "fwd"))
def test_golden_examples(case):
    chars, rc, off, want, bad = case
    got, n_bad = O.pack(_chars(chars), off, revcomp=rc)
    assert got.tobytes() == want
    assert n_bad == bad


def _check_forward(pack, seed):
    seqs, off = _reads(seed, 60, 70)
    text = "".join(seqs)
    mixed = "".join(c.lower() if i % 3 == 0 else c for i, c in enumerate(text))
    got, bad = pack(_chars(mixed), off, False)
    ref = _gen_pack(seqs)
    nb = (len(text) + 3) // 4
    return bad == 0 and got.size == ((len(text) + 15) // 16) * 4 and \
        got[:nb].tobytes() == ref[:nb].tobytes() and not got[nb:].any()


def _check_revcomp(pack, seed):
    seqs, off = _reads(seed, 60, 70)
    got, bad = pack(_chars("".join(seqs)), off, True)
    rcs = [s[::-1].translate(RC) for s in seqs]
    ref = _gen_pack(rcs)
    nb = (int(off[-1]) + 3) // 4
    return bad == 0 and got[:nb].tobytes() == ref[:nb].tobytes()


def _check_invalid(pack, seed):
    rng = random.Random(seed)
    text = "".join(rng.choice("ACGTNacgtn-X") for _ in range(301))
    n_bad = sum(c not in "ACGTacgt" for c in text)
    clean = "".join(c if c in "ACGTacgt" else "A" for c in text)
    got, bad = pack(_chars(text), np.array([0, len(text)], np.int64), False)
    ref = _gen_pack([clean])
    nb = (len(text) + 3) // 4
    return bad == n_bad and got[:nb].tobytes() == ref[:nb].tobytes()


def _oracle_pack(chars, off, rc):
    return O.pack(chars, off, revcomp=rc)


def test_forward_matches_generator_packer():
    for seed in range(5):
        assert _check_forward(_oracle_pack, seed)


def test_revcomp_matches_string_definition():
    for seed in range(5):
        assert _check_revcomp(_oracle_pack, seed)


def test_invalid_bases_are_counted_and_zeroed():
    for seed in range(3):
        assert _check_invalid(_oracle_pack, seed)


def test_revcomp_twice_is_identity():
    seqs, off = _reads(9, 40, 50)
    once = [s[::-1].translate(RC) for s in seqs]
    got, _ = O.pack(_chars("".join(once)), off, revcomp=True)
    fwd, _ = O.pack(_chars("".join(seqs)), off, revcomp=False)
    assert got.tobytes() == fwd.tobytes()


def test_pack_then_align_equals_align():
    q, qo = _reads(3, 50, 60)
    t, to = _reads(4, 50, 80)
    qp, _ = O.pack(_chars("".join(q)), qo)
    tp, _ = O.pack(_chars("".join(t)), to)
    got = O.align_batch(qp, qo, tp, to)
    b = I.from_strings(q, t)
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


MUTANTS = {
    "no_complement": ("if (ok) code = 3 - code;", "(void)0;"),
    "msb_first": ("out[k >> 2] |= (uint8_t)(code << (2 * (k & 3)));",
                  "out[k >> 2] |= (uint8_t)(code << (6 - 2 * (k & 3)));"),
    "mirror_off_by_one": ("off[s] + off[s + 1] - 1 - k", "off[s] + off[s + 1] - k"),
    "mirror_whole_stream": ("src = off[s] + off[s + 1] - 1 - k;",
                            "src = off[n_seqs] - 1 - k;"),
    "upper_case_only": ("case 'A': case 'a':", "case 'A':"),
    "invalid_not_counted": ("++invalid;\n            code = 0;", "code = 0;"),
    "g_and_c_swapped": ("case 'C': case 'c': *code = 1;", "case 'C': case 'c': *code = 2;"),
}


def _build_mutant(text, tmp, name):
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", so, c], check=True)
    lib = ctypes.CDLL(so)
    p, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_pack.argtypes = [p, i64, p, i64, ctypes.c_int, p]
    lib.oracle_pack.restype = i64

    def pack(chars, off, rc):
        chars = np.ascontiguousarray(chars, np.uint8)
        off = np.ascontiguousarray(off, np.int64)
        out = np.zeros(((chars.size + 15) // 16) * 4, np.uint8)
        bad = lib.oracle_pack(chars.ctypes.data, chars.size, off.ctypes.data, off.size - 1,
                              1 if rc else 0, out.ctypes.data)
        return out, bad
    return pack


def _passes_all(pack):
    if not all(_check_forward(pack, s) for s in range(2)):
        return False
    if not all(_check_revcomp(pack, s) for s in range(2)):
        return False
    if not _check_invalid(pack, 0):
        return False
    for chars, rc, off, want, bad in _golden():
        got, n_bad = pack(_chars(chars), off, rc)
        if got.tobytes() != want or n_bad != bad:
            return False
    return True


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site moved: %s" % name
    with tempfile.TemporaryDirectory() as tmp:
        assert _passes_all(_build_mutant(src, tmp, "real"))
        assert not _passes_all(_build_mutant(src.replace(old, new), tmp, name))
