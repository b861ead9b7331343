"""Seeded synthetic workloads and the 2-bit packed input format.

This module holds no alignment arithmetic.  It only draws random sequences
and packs them, so both the GPU path's tests/benchmarks and the CPU oracle
can be fed the same bytes.

Format (the library's input convention): bases A=0, C=1, G=2, T=3; base k of
a stream sits in byte k>>2 at bits 2*(k&3) (least-significant pair first).
A batch is two independent streams (queries and targets) plus int64 CSR
offsets in bases: pair p is query [q_off[p], q_off[p+1]) against target
[t_off[p], t_off[p+1]).  Pair starts are not byte aligned.

Workloads stand in for the paper's inputs (Section V-B synthetic reads of
64-4096 bp from a Wgsim-like simulator; Section V-D BWA-MEM seeds of
Illumina 250 bp reads and PacBio reads of ~2 kbp).  The real datasets are
not used; every sequence here is drawn from numpy's PCG64 generator.

Mutation model used by every workload: each source base independently is
  substituted (probability p_sub, the new base uniform over the other 3),
  deleted (p_indel/2, removing a run of L source bases), or
  followed by an insertion (p_indel/2, L fresh random bases),
with L = 1 for single-base indels or L ~ Geometric(1/2) (mean 2).
"""
from __future__ import annotations

import hashlib
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

GENERATOR_VERSION = "salo-inputs-1"
BASES = "ACGT"


# ----------------------------------------------------------------- packing

def pack_bases(codes: np.ndarray) -> np.ndarray:
    """Pack a uint8 array of base codes (0..3) into 2-bit LSB-first bytes.

    The result is padded with zero bytes to a multiple of 4 bytes plus 4,
    so 32-bit word reads at the tail stay inside the buffer.
    """
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    n = codes.size
    nbytes = (n + 3) // 4
    padded = np.zeros(nbytes * 4, dtype=np.uint8)
    padded[:n] = codes & 3
    quads = padded.reshape(-1, 4)
    packed = (quads[:, 0] | (quads[:, 1] << 2) | (quads[:, 2] << 4)
              | (quads[:, 3] << 6)).astype(np.uint8)
    total = ((nbytes + 3) // 4) * 4 + 4
    out = np.zeros(total, dtype=np.uint8)
    out[:nbytes] = packed
    return out


def unpack_bases(packed: np.ndarray, start: int, length: int) -> np.ndarray:
    """Return base codes [start, start+length) of a packed stream."""
    k = np.arange(start, start + length, dtype=np.int64)
    return ((packed[k >> 2] >> (2 * (k & 3)).astype(np.uint8)) & 3).astype(np.uint8)


def encode(s: str) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for i, c in enumerate(BASES):
        lut[ord(c)] = i
        lut[ord(c.lower())] = i
    a = lut[np.frombuffer(s.encode(), dtype=np.uint8)]
    if np.any(a == 255):
        raise ValueError("only A, C, G, T are allowed")
    return a


def decode(codes: np.ndarray) -> str:
    return "".join(BASES[int(c)] for c in codes)


@dataclass
class Batch:
    """A packed batch: the exact arrays handed to the library and oracle."""
    q_seqs: np.ndarray      # uint8, packed
    q_offsets: np.ndarray   # int64 [n+1]
    t_seqs: np.ndarray      # uint8, packed
    t_offsets: np.ndarray   # int64 [n+1]
    name: str = ""

    @property
    def n_pairs(self) -> int:
        return len(self.q_offsets) - 1

    def q_lens(self) -> np.ndarray:
        return np.diff(self.q_offsets)

    def t_lens(self) -> np.ndarray:
        return np.diff(self.t_offsets)

    def cells(self) -> int:
        return int(np.sum(self.q_lens().astype(np.int64) * self.t_lens()))

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.q_seqs, self.q_offsets, self.t_seqs, self.t_offsets):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def pair_strings(self, p: int):
        q0, q1 = int(self.q_offsets[p]), int(self.q_offsets[p + 1])
        t0, t1 = int(self.t_offsets[p]), int(self.t_offsets[p + 1])
        return (decode(unpack_bases(self.q_seqs, q0, q1 - q0)),
                decode(unpack_bases(self.t_seqs, t0, t1 - t0)))

    def subset(self, idx) -> "Batch":
        """A new batch holding pairs idx (in that order), repacked."""
        idx = np.asarray(idx, dtype=np.int64)
        ql = self.q_lens()[idx]
        tl = self.t_lens()[idx]
        qs = _gather_stream(self.q_seqs, self.q_offsets[idx], ql)
        ts = _gather_stream(self.t_seqs, self.t_offsets[idx], tl)
        return Batch(pack_bases(qs), _offsets(ql), pack_bases(ts), _offsets(tl),
                     name=self.name + "[subset]")


def _offsets(lens: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def _gather_stream(packed, starts, lens) -> np.ndarray:
    total = int(np.sum(lens))
    if total == 0:
        return np.zeros(0, np.uint8)
    grp_start = np.repeat(np.asarray(starts, np.int64) - _offsets(lens)[:-1], lens)
    k = np.arange(total, dtype=np.int64) + grp_start
    return ((packed[k >> 2] >> (2 * (k & 3)).astype(np.uint8)) & 3).astype(np.uint8)


def from_strings(queries, targets, name="strings") -> Batch:
    """Build a batch from Python strings over ACGT."""
    if len(queries) != len(targets):
        raise ValueError("need one target per query")
    qc = [encode(s) for s in queries]
    tc = [encode(s) for s in targets]
    ql = np.array([len(a) for a in qc], np.int64)
    tl = np.array([len(a) for a in tc], np.int64)
    qs = np.concatenate(qc) if qc else np.zeros(0, np.uint8)
    ts = np.concatenate(tc) if tc else np.zeros(0, np.uint8)
    return Batch(pack_bases(qs), _offsets(ql), pack_bases(ts), _offsets(tl), name)


def from_codes(q_list, t_list, name="codes") -> Batch:
    ql = np.array([len(a) for a in q_list], np.int64)
    tl = np.array([len(a) for a in t_list], np.int64)
    qs = np.concatenate(q_list).astype(np.uint8) if len(q_list) else np.zeros(0, np.uint8)
    ts = np.concatenate(t_list).astype(np.uint8) if len(t_list) else np.zeros(0, np.uint8)
    return Batch(pack_bases(qs), _offsets(ql), pack_bases(ts), _offsets(tl), name)


# ---------------------------------------------------------------- mutation

def _mutate(rng, src: np.ndarray, src_lens: np.ndarray, p_sub: float,
            p_indel: float, geometric: bool):
    """Apply the mutation model to a concatenation of sources.

    Returns (stream, lens): the mutated concatenation and per-source lengths.
    Events are sparse, so only event positions are touched.
    """
    total = src.size
    n = len(src_lens)
    if total == 0:
        return src.copy(), np.zeros(n, np.int64)
    src_off = _offsets(src_lens)
    u = rng.random(total, dtype=np.float32)
    ev = np.flatnonzero(u < np.float32(p_sub + p_indel))
    uev = u[ev]
    p_del = p_indel / 2.0
    sub = ev[uev < np.float32(p_sub)]
    dele = ev[(uev >= np.float32(p_sub)) & (uev < np.float32(p_sub + p_del))]
    ins = ev[uev >= np.float32(p_sub + p_del)]
    mutated = src.copy()
    if sub.size:
        mutated[sub] = (src[sub] + rng.integers(1, 4, sub.size, dtype=np.uint8)) & 3
    if geometric:
        dl = rng.geometric(0.5, dele.size).astype(np.int64)
        il = rng.geometric(0.5, ins.size).astype(np.int64)
    else:
        dl = np.ones(dele.size, np.int64)
        il = np.ones(ins.size, np.int64)
    # deletion runs [p, min(p+L, end of its source))
    d_pair = np.searchsorted(src_off, dele, side="right") - 1
    d_end = np.minimum(dele + dl, src_off[d_pair + 1])
    run = d_end - dele
    nrun = int(run.sum())
    if nrun:
        delpos = np.repeat(dele - (np.cumsum(run) - run), run) + np.arange(nrun)
        delpos = np.unique(delpos)
    else:
        delpos = np.zeros(0, np.int64)
    # insertions: il fresh bases right after source position p
    ins_idx = np.repeat(ins + 1, il)
    out = np.insert(mutated, ins_idx, _rand_bases(rng, ins_idx.size))
    if delpos.size:
        shift = np.searchsorted(ins_idx, delpos, side="right")
        out = np.delete(out, delpos + shift)
    lens = src_lens.astype(np.int64).copy()
    if delpos.size:
        lens -= np.bincount(np.searchsorted(src_off, delpos, side="right") - 1,
                            minlength=n)
    if ins.size:
        i_pair = np.searchsorted(src_off, ins, side="right") - 1
        lens += np.bincount(i_pair, weights=il, minlength=n).astype(np.int64)
    return out, lens


def _rand_bases(rng, n):
    return rng.integers(0, 4, int(n), dtype=np.uint8)


def _assemble(q_parts, t_parts):
    """Concatenate per-chunk (stream, lens) lists into one packed Batch."""
    qs = np.concatenate([p[0] for p in q_parts]) if q_parts else np.zeros(0, np.uint8)
    ql = np.concatenate([p[1] for p in q_parts]) if q_parts else np.zeros(0, np.int64)
    ts = np.concatenate([p[0] for p in t_parts]) if t_parts else np.zeros(0, np.uint8)
    tl = np.concatenate([p[1] for p in t_parts]) if t_parts else np.zeros(0, np.int64)
    return Batch(pack_bases(qs), _offsets(ql), pack_bases(ts), _offsets(tl))


def _place_source(rng, src_lens, t_lens):
    """Targets = random left flank + source + random right flank."""
    flank = t_lens - src_lens
    left = (rng.random(len(src_lens)) * (flank + 1)).astype(np.int64)
    left = np.minimum(left, flank)
    right = flank - left
    return left, right


def _build_targets(rng, src, src_lens, left, right):
    """t = left flank + source + right flank, vectorised over pairs."""
    n = len(src_lens)
    tl = left + src_lens + right
    total = int(tl.sum())
    t = _rand_bases(rng, total)
    t_off = _offsets(tl)
    s_off = _offsets(src_lens)
    # copy each source into its slot after the left flank
    if src.size:
        dst_start = np.repeat(t_off[:-1] + left - s_off[:-1], src_lens)
        t[np.arange(src.size, dtype=np.int64) + dst_start] = src
    return t, tl


# ---------------------------------------------------------------- workloads

CHUNK_PAIRS = 100_000   # part of the generator definition (fixes the seeds)


def _chunked(n_pairs: int, make, progress=None, workers: int = 0):
    """Run make(c0, n) for every chunk of CHUNK_PAIRS pairs and assemble the
    parts in chunk order.  Each chunk draws from its own seeded generator,
    so the batch is the same whatever the number of worker threads (numpy
    releases the interpreter lock in its bulk loops)."""
    starts = list(range(0, n_pairs, CHUNK_PAIRS))
    if workers <= 0:
        workers = min(8, os.cpu_count() or 1)
    parts = [None] * len(starts)

    def one(k):
        c0 = starts[k]
        parts[k] = make(c0, min(CHUNK_PAIRS, n_pairs - c0))

    if workers == 1 or len(starts) <= 1:
        for k, c0 in enumerate(starts):
            if progress is not None:
                progress(c0, n_pairs)
            one(k)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for k, _ in enumerate(ex.map(one, range(len(starts)))):
                if progress is not None:
                    progress(starts[k], n_pairs)
    return _assemble([p[0] for p in parts], [p[1] for p in parts])


def plain_small(seed: int = 0, n_pairs: int = 1000) -> Batch:
    """Parity workload: 1,000 pairs; target = 250 random bases; query = 150
    bases emitted by walking the target from a uniform start in [0, 90]
    with 2% substitutions and 0.5% single-base indels."""
    rng = np.random.default_rng([seed, 1])
    tlen, qlen = 250, 150
    t = _rand_bases(rng, n_pairs * tlen).reshape(n_pairs, tlen)
    start = rng.integers(0, 91, n_pairs)
    src_lens = (tlen - start).astype(np.int64)
    src = np.concatenate([t[p, start[p]:] for p in range(n_pairs)])
    mq, ml = _mutate(rng, src, src_lens, 0.02, 0.005, geometric=False)
    mo = _offsets(ml)
    q = np.empty((n_pairs, qlen), np.uint8)
    for p in range(n_pairs):
        seg = mq[mo[p]:mo[p + 1]][:qlen]
        if seg.size < qlen:   # the walk ran out of source: continue at random
            seg = np.concatenate([seg, _rand_bases(rng, qlen - seg.size)])
        q[p] = seg
    b = Batch(pack_bases(q.reshape(-1)), _offsets(np.full(n_pairs, qlen, np.int64)),
              pack_bases(t.reshape(-1)), _offsets(np.full(n_pairs, tlen, np.int64)))
    b.name = "plain_small"
    return b


def short_reads(seed: int = 0, n_pairs: int = 2_000_000, progress=None,
                workers: int = 0) -> Batch:
    """Short-read extension: source length U{50..250}; target = source plus
    a U{0..100} flank split at random into left/right; query = source with
    1% substitutions and 0.1% single-base indels; 10% of pairs are
    unrelated random sequences of the same lengths."""
    def chunk(c0, n):
        rng = np.random.default_rng([seed, 2, c0 // CHUNK_PAIRS])
        src_lens = rng.integers(50, 251, n).astype(np.int64)
        flank = rng.integers(0, 101, n).astype(np.int64)
        left, right = _place_source(rng, src_lens, src_lens + flank)
        unrelated = rng.random(n) < 0.10
        src = _rand_bases(rng, src_lens.sum())
        t, tl = _build_targets(rng, src, src_lens, left, right)
        mq, ml = _mutate(rng, src, src_lens, 0.01, 0.001, geometric=False)
        # unrelated pairs: replace query and target by fresh random bases
        if unrelated.any():
            qo, to = _offsets(ml), _offsets(tl)
            qmask = np.repeat(unrelated, ml)
            tmask = np.repeat(unrelated, tl)
            mq = mq.copy()
            mq[qmask] = _rand_bases(rng, qmask.sum())
            t[tmask] = _rand_bases(rng, tmask.sum())
            del qo, to
        return (mq, ml), (t, tl)

    b = _chunked(n_pairs, chunk, progress, workers)
    b.name = "short_reads"
    return b


def long_uneven(seed: int = 0, n_pairs: int = 200_000, progress=None,
                workers: int = 0) -> Batch:
    """Long uneven extension: source length round(exp(U[ln 500, ln 5000]));
    target length round(source * U[1.1, 1.5]) with the source at a random
    offset; query = source with 5% substitutions and 3% indels of geometric
    length (mean 2)."""
    def chunk(c0, n):
        rng = np.random.default_rng([seed, 3, c0 // CHUNK_PAIRS])
        src_lens = np.rint(np.exp(rng.uniform(np.log(500), np.log(5000), n))).astype(np.int64)
        tl = np.rint(src_lens * rng.uniform(1.1, 1.5, n)).astype(np.int64)
        left, right = _place_source(rng, src_lens, tl)
        src = _rand_bases(rng, src_lens.sum())
        t, tl = _build_targets(rng, src, src_lens, left, right)
        mq, ml = _mutate(rng, src, src_lens, 0.05, 0.03, geometric=True)
        return (mq, ml), (t, tl)

    b = _chunked(n_pairs, chunk, progress, workers)
    b.name = "long_uneven"
    return b


def anchored_long(seed: int = 0, n_pairs: int = 200_000, progress=None,
                  workers: int = 0) -> Batch:
    """Anchored long extension, the input of banded extension: the long
    uneven workload's lengths and error model (source length
    round(exp(U[ln 500, ln 5000])), target length round(source *
    U[1.1, 1.5]), 5% substitutions, 3% indels of geometric length, mean 2),
    but with the source at target offset 0, as when both sequences start at
    the end of a seed: the best path starts near cell (0, 0) and stays near
    the main diagonal."""
    def chunk(c0, n):
        rng = np.random.default_rng([seed, 6, c0 // CHUNK_PAIRS])
        src_lens = np.rint(np.exp(rng.uniform(np.log(500), np.log(5000), n))).astype(np.int64)
        tl = np.rint(src_lens * rng.uniform(1.1, 1.5, n)).astype(np.int64)
        left = np.zeros(n, np.int64)
        right = tl - src_lens
        src = _rand_bases(rng, src_lens.sum())
        t, tl = _build_targets(rng, src, src_lens, left, right)
        mq, ml = _mutate(rng, src, src_lens, 0.05, 0.03, geometric=True)
        return (mq, ml), (t, tl)

    b = _chunked(n_pairs, chunk, progress, workers)
    b.name = "anchored_long"
    return b


def band_cells(q_lens, t_lens, band: int) -> np.ndarray:
    """Per pair, the number of cells (i, j), 0 <= i < t_len, 0 <= j < q_len,
    with |i - j| <= band: the sum over diagonals d = j - i of their length."""
    q_lens = np.asarray(q_lens, np.int64)
    t_lens = np.asarray(t_lens, np.int64)
    total = np.zeros(q_lens.shape, np.int64)
    for d in range(-band, band + 1):
        lo = max(0, -d)
        total += np.maximum(0, np.minimum(t_lens, q_lens - d) - lo)
    return total


def mixed(seed: int = 0, n_pairs: int = 4_000_000, progress=None,
          workers: int = 0) -> Batch:
    """Batched mixed workload: source length drawn from a mixture of
    60% U{100..300}, 35% U{300..1000}, 5% U{1000..10000}; target length
    round(1.2 * source) with the source at a random offset; query = source
    with 2% substitutions and 1% single-base indels."""
    def chunk(c0, n):
        rng = np.random.default_rng([seed, 4, c0 // CHUNK_PAIRS])
        src_lens = mixed_lengths(rng, n)
        tl = np.rint(1.2 * src_lens).astype(np.int64)
        left, right = _place_source(rng, src_lens, tl)
        src = _rand_bases(rng, src_lens.sum())
        t, tl = _build_targets(rng, src, src_lens, left, right)
        mq, ml = _mutate(rng, src, src_lens, 0.02, 0.01, geometric=False)
        return (mq, ml), (t, tl)

    b = _chunked(n_pairs, chunk, progress, workers)
    b.name = "mixed"
    return b


def mixed_lengths(rng, n):
    u = rng.random(n)
    a = rng.integers(100, 301, n)
    b = rng.integers(300, 1001, n)
    c = rng.integers(1000, 10001, n)
    return np.where(u < 0.60, a, np.where(u < 0.95, b, c)).astype(np.int64)


def random_n_masks(q_total: int, t_total: int, fraction: float, seed: int = 0):
    """Seeded N masks for a batch's two streams: each base is marked N with
    probability `fraction`, drawn for the query stream first and then for
    the target stream from one generator.  Returns two uint32 arrays of one
    bit per base (bit k of word k >> 5), the layout the N-mask calls take."""
    rng = np.random.default_rng([seed, 99])

    def one(total):
        bits = rng.random(total) < fraction
        words = np.zeros(max((total + 31) // 32, 1), np.uint32)
        idx = np.nonzero(bits)[0]
        np.bitwise_or.at(words, idx >> 5, np.uint32(1) << (idx & 31).astype(np.uint32))
        return words
    qm = one(int(q_total))
    return qm, one(int(t_total))


def random_pairs(seed: int, n_pairs: int, max_len: int, min_len: int = 0,
                 related: float = 0.5) -> Batch:
    """Fuzz workload: independent lengths U{min_len..max_len}; a fraction of
    pairs are related (query = mutated window of the target)."""
    rng = np.random.default_rng([seed, 5])
    ql = rng.integers(min_len, max_len + 1, n_pairs).astype(np.int64)
    tl = rng.integers(min_len, max_len + 1, n_pairs).astype(np.int64)
    qs, ts = [], []
    for p in range(n_pairs):
        t = _rand_bases(rng, tl[p])
        if rng.random() < related and tl[p] > 0 and ql[p] > 0:
            s0 = int(rng.integers(0, tl[p]))
            src = t[s0:s0 + ql[p]]
            m, _ = _mutate(rng, src, np.array([src.size]), 0.05, 0.03, True)
            q = np.concatenate([m, _rand_bases(rng, max(0, ql[p] - m.size))])[:ql[p]]
        else:
            q = _rand_bases(rng, ql[p])
        qs.append(q)
        ts.append(t)
    b = from_codes(qs, ts)
    b.name = "random_pairs"
    return b


WORKLOADS = {
    "plain_small": plain_small,
    "short_reads": short_reads,
    "long_uneven": long_uneven,
    "mixed": mixed,
    "anchored_long": anchored_long,
}
