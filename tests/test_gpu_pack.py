"""GPU packing kernels (salo_pack_bases) against the packing oracle,
bit for bit, forward and reverse-complemented, with the invalid-base
count; and pack-then-align on the GPU against the alignment oracle."""
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_09310_amd import inputs as I

pytestmark = pytest.mark.gpu
LETTERS = np.frombuffer(b"ACGT", np.uint8)


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


def _gpu_pack(chars, off, rc, shift=0):
    import torch
    from paper_2301_09310_amd import salo
    c = torch.from_numpy(np.ascontiguousarray(chars, np.uint8)).cuda()
    if shift:
        # a view `shift` bytes into a larger buffer: 4-byte aligned, not 16
        buf = torch.zeros(chars.size + 16, dtype=torch.uint8, device="cuda")
        buf[shift:shift + chars.size] = c
        c = buf[shift:shift + chars.size]
    o = torch.from_numpy(np.ascontiguousarray(off, np.int64)).cuda()
    inv = torch.zeros(1, dtype=torch.int64, device="cuda")
    # output buffer pre-filled with garbage: every byte must be written
    nbytes = ((chars.size + 15) // 16) * 4
    out = torch.full((max(nbytes, 4),), 0xA5, dtype=torch.uint8, device="cuda")
    salo.pack_bases(c, o, revcomp=rc, out=out, invalid=inv)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:nbytes], int(inv.item())


def _check(chars, off, label, shift=0):
    for rc in (False, True):
        _say(label, "revcomp" if rc else "forward", "n_chars", chars.size, "n_seqs",
             off.size - 1, "shift", shift)
        got, bad = _gpu_pack(chars, off, rc, shift)
        want, wbad = O.pack(chars, off, revcomp=rc)
        diff = np.nonzero(got != want)[0]
        assert diff.size == 0, "%s rc=%s: first differing byte %d gpu %02x oracle %02x" % (
            label, rc, diff[0], got[diff[0]], want[diff[0]])
        assert bad == wbad, (label, rc, bad, wbad)


def _random_case(seed, n_seqs, max_len, noise=0.0):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n_seqs)
    off = np.zeros(n_seqs + 1, np.int64)
    off[1:] = np.cumsum(lens)
    chars = LETTERS[rng.integers(0, 4, int(off[-1]))]
    lower = rng.random(chars.size) < 0.3
    chars = np.where(lower, chars | 0x20, chars).astype(np.uint8)
    if noise:
        bad = rng.random(chars.size) < noise
        chars = np.where(bad, np.frombuffer(b"N", np.uint8)[0], chars).astype(np.uint8)
    return chars, off


def test_ragged_lengths(dev):
    for total in [1, 2, 15, 16, 17, 31, 32, 33, 4095, 4096, 4097, 65537]:
        rng = np.random.default_rng(total)
        chars = LETTERS[rng.integers(0, 4, total)]
        cut = np.sort(rng.integers(0, total + 1, 5))
        off = np.concatenate([[0], cut, [total]]).astype(np.int64)
        _check(chars, off, "total %d" % total)


def test_random_reads_with_invalid_bases(dev):
    chars, off = _random_case(1, 5000, 300, noise=0.01)
    _check(chars, off, "random reads, 1% N")


def test_many_tiny_sequences(dev):
    """More than 1024 sequences inside one reverse-complement block's 32,768
    bases (lengths 0..3): the staged offset window runs out and the kernel
    searches the offsets in global memory."""
    chars, off = _random_case(2, 20000, 3)
    _check(chars, off, "tiny sequences")


def test_block_boundaries_and_empty_runs(dev):
    """Sequence bounds on the reverse-complement blocks' edges (multiples of
    32,768 bases) and next to them; a run of empty sequences (several
    sequences mark the same word in a block's table of word sequences); and
    1,200 two-base sequences, more than one block's window of staged
    offsets holds."""
    rng = np.random.default_rng(17)
    block = 32768
    cuts = [k * block + d for k in range(1, 6) for d in (-17, -16, -1, 0, 1, 15, 16)]
    cuts += list(rng.integers(0, 6 * block, 300))
    cuts += [2 * block + 5] * 7
    cuts += list(4 * block + 100 + np.arange(0, 2400, 2))
    total = 6 * block + 123
    off = np.concatenate([[0], np.sort(np.array(cuts, np.int64)), [total]]).astype(np.int64)
    chars = LETTERS[rng.integers(0, 4, total)]
    _check(chars, off, "block edges")


def test_single_long_sequence(dev):
    chars, off = _random_case(3, 1, 200000)
    _check(chars, off, "one long sequence")


def test_short_reads_ascii(dev):
    """200,000 short-read pairs written out as characters, both streams."""
    b = I.short_reads(0, 200_000)
    for name, packed, off in (("queries", b.q_seqs, b.q_offsets), ("targets", b.t_seqs, b.t_offsets)):
        n = int(off[-1])
        codes = (np.unpackbits(packed[: (n + 3) // 4, None], axis=1, bitorder="little")
                 .reshape(-1, 4, 2) @ np.array([1, 2], np.uint8)).reshape(-1)[:n]
        _check(LETTERS[codes], off, "short_reads " + name)


def test_pack_then_align(dev):
    """Characters packed on the GPU (forward, and reverse-complemented back
    from their reverse complements) align exactly like the oracle packing."""
    import torch
    from paper_2301_09310_amd import salo
    rng = random.Random(5)
    q = ["".join(rng.choice("ACGTacgt") for _ in range(rng.randint(0, 300))) for _ in range(800)]
    t = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 400))) for _ in range(800)]
    rc = str.maketrans("ACGTacgt", "TGCAtgca")
    t_rc = [s[::-1].translate(rc) for s in t]        # packed back with revcomp
    qo = np.zeros(801, np.int64); qo[1:] = np.cumsum([len(s) for s in q])
    to = np.zeros(801, np.int64); to[1:] = np.cumsum([len(s) for s in t])
    qc = torch.from_numpy(np.frombuffer("".join(q).encode(), np.uint8).copy()).cuda()
    tc = torch.from_numpy(np.frombuffer("".join(t_rc).encode(), np.uint8).copy()).cuda()
    qo_d, to_d = torch.from_numpy(qo).cuda(), torch.from_numpy(to).cuda()
    qp = salo.pack_bases(qc, qo_d)
    tp = salo.pack_bases(tc, to_d, revcomp=True)
    res = salo.align_batch(qp, qo_d, tp, to_d)
    torch.cuda.synchronize()
    b = I.from_strings([s.upper() for s in q], t)
    want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets)
    for g, w, name in zip(res, want, ("score", "q_end", "t_end")):
        assert np.array_equal(g.cpu().numpy().astype(np.int64), w), name


@pytest.mark.parametrize("shift", [4, 8, 12])
def test_buffer_not_16_byte_aligned(dev, shift):
    """The dword-gather kernels (a character buffer that is 4- but not
    16-byte aligned) against the oracle, on ragged reads with invalid bases."""
    chars, off = _random_case(91 + shift, 500, 400, noise=0.02)
    _check(chars, off, "unaligned", shift=shift)
