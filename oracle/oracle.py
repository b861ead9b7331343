"""CPU oracle for batched affine-gap seed extension -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path (the HIP library and its binding)
never imports, links or calls it.

It wraps ``gotoh_oracle.c``: a plain scalar int64 implementation of the
SALoBa paper's Eq. 1 (Section II-A), the affine-gap Smith-Waterman-Gotoh
recurrence, returning per pair the highest cell score and its end position
(first maximum in row-major order over target rows and query columns; see
the header of the C file for every reading of the paper it takes), and the
companion files: ``pack_oracle.c`` (2-bit packing and reverse complement),
``start_oracle.c`` (start positions of the best alignment) and
``band_oracle.c`` (Eq. 1 restricted to a diagonal band, Section VII-B) and
``trace_oracle.c`` (the optimal path between start and end, as a CIGAR).

The shared library is compiled from the C source with gcc on first use
(and by the repository's build step); it has no dependency on the GPU code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gotoh_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "pack_oracle.c"), os.path.join(_HERE, "start_oracle.c"),
         os.path.join(_HERE, "band_oracle.c"), os.path.join(_HERE, "trace_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle_gotoh.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (-O2, plain scalar C)."""
    if (not force and os.path.exists(_LIB)
            and all(os.path.getmtime(_LIB) >= os.path.getmtime(f) for f in _SRCS)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
           "-o", tmp] + _SRCS
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64 = ctypes.c_int64
            p = ctypes.c_void_p
            lib.oracle_align_batch.argtypes = [p, p, p, p, i64, i64, i64, i64,
                                               i64, p, p, p, ctypes.c_int]
            lib.oracle_align_batch.restype = ctypes.c_int
            lib.oracle_cell_h.argtypes = [p, i64, i64, p, i64, i64, i64, i64,
                                          i64, i64, i64, i64]
            lib.oracle_cell_h.restype = i64
            lib.oracle_pack.argtypes = [p, i64, p, i64, ctypes.c_int, p]
            lib.oracle_pack.restype = i64
            lib.oracle_pack_n.argtypes = [p, i64, p, i64, ctypes.c_int, p, p]
            lib.oracle_pack_n.restype = i64
            lib.oracle_align_batch_n.argtypes = [p, p, p, p, p, p, i64, i64, i64, i64, i64,
                                                 p, p, p, ctypes.c_int]
            lib.oracle_align_batch_n.restype = ctypes.c_int
            lib.oracle_start_batch_n.argtypes = [p, p, p, p, p, p, i64, i64, i64, i64, i64,
                                                 p, p, p, p, p]
            lib.oracle_start_batch_n.restype = i64
            lib.oracle_align_banded.argtypes = [p, p, p, p, i64, i64, i64, i64, i64, i64,
                                                p, p, p]
            lib.oracle_align_banded.restype = ctypes.c_int
            lib.oracle_trace_batch.argtypes = [p, p, p, p, i64, i64, i64, i64, i64,
                                               p, p, p, p, p, p, p, p]
            lib.oracle_trace_batch.restype = i64
            lib.oracle_start_batch.argtypes = [p, p, p, p, i64, i64, i64, i64, i64,
                                               p, p, p, p, p]
            lib.oracle_start_batch.restype = i64
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _mask_ptr(mask, n_bases):
    """(address or None, array kept alive) of an optional N mask."""
    if mask is None:
        return None, None
    m = np.ascontiguousarray(mask, dtype=np.uint32)
    if m.size * 32 < int(n_bases):
        raise ValueError("N mask shorter than the stream")
    if m.size == 0:
        m = np.zeros(1, np.uint32)
    return m.ctypes.data, m


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def align_batch(q_seqs, q_offsets, t_seqs, t_offsets, scoring=(1, -4, 6, 1),
                nthreads: int | None = None, q_nmask=None, t_nmask=None):
    """Oracle alignment of every pair.

    q_seqs/t_seqs: uint8 arrays of 2-bit packed bases (4 per byte, LSB first).
    q_offsets/t_offsets: int64 arrays of length n_pairs+1 (CSR, in bases).
    scoring: (match, mismatch, gap_open, gap_extend); a gap of k bases costs
    gap_open + k*gap_extend.
    q_nmask/t_nmask: optional uint32 arrays, bit k of word k>>5 marking base
    k of the stream as N (an N scores mismatch against every base).
    Returns (score, q_end, t_end) as int64 arrays.
    """
    lib = _load()
    q_seqs = np.ascontiguousarray(q_seqs, dtype=np.uint8)
    t_seqs = np.ascontiguousarray(t_seqs, dtype=np.uint8)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.int64)
    t_offsets = np.ascontiguousarray(t_offsets, dtype=np.int64)
    n = len(q_offsets) - 1
    if n < 0 or len(t_offsets) != n + 1:
        raise ValueError("offset arrays must both have n_pairs+1 entries")
    if n and (np.any(np.diff(q_offsets) < 0) or np.any(np.diff(t_offsets) < 0)):
        raise ValueError("offsets must be non-decreasing")
    if n and (q_offsets[-1] > 4 * len(q_seqs) or t_offsets[-1] > 4 * len(t_seqs)):
        raise ValueError("offsets run past the packed buffers")
    score = np.zeros(max(n, 0), dtype=np.int64)
    qend = np.zeros(max(n, 0), dtype=np.int64)
    tend = np.zeros(max(n, 0), dtype=np.int64)
    if n == 0:
        return score, qend, tend
    # empty buffers still need a valid address
    qb = q_seqs if len(q_seqs) else np.zeros(1, np.uint8)
    tb = t_seqs if len(t_seqs) else np.zeros(1, np.uint8)
    a, b, o, e = (int(x) for x in scoring)
    qm = _mask_ptr(q_nmask, q_offsets[-1])
    tm = _mask_ptr(t_nmask, t_offsets[-1])
    rc = lib.oracle_align_batch_n(_ptr(qb), qm[0], _ptr(q_offsets), _ptr(tb), tm[0],
                                  _ptr(t_offsets), n, a, b, o, e, _ptr(score),
                                  _ptr(qend), _ptr(tend),
                                  int(nthreads or default_threads()))
    if rc != 0:
        raise MemoryError("oracle_align_batch failed (%d)" % rc)
    return score, qend, tend


def cell_h(q_seqs, q_start, m, t_seqs, t_start, n, scoring, ti, qj) -> int:
    """H(ti, qj) of one pair's table (Eq. 1), or -1 outside the table."""
    lib = _load()
    q_seqs = np.ascontiguousarray(q_seqs, dtype=np.uint8)
    t_seqs = np.ascontiguousarray(t_seqs, dtype=np.uint8)
    a, b, o, e = (int(x) for x in scoring)
    return int(lib.oracle_cell_h(_ptr(q_seqs), int(q_start), int(m),
                                 _ptr(t_seqs), int(t_start), int(n),
                                 a, b, o, e, int(ti), int(qj)))


def align_strings(q: str, t: str, scoring=(1, -4, 6, 1)):
    """Convenience for tests: align two ACGT strings, return (score, qend, tend)."""
    qs, qo = _pack_strings([q])
    ts, to = _pack_strings([t])
    s, qe, te = align_batch(qs, qo, ts, to, scoring, nthreads=1)
    return int(s[0]), int(qe[0]), int(te[0])


def _pack_strings(seqs):
    """Local 2-bit packer used only by align_strings (the oracle keeps its
    own copy of the input convention; it shares no code with the generator)."""
    code = {"A": 0, "C": 1, "G": 2, "T": 3}
    bases = [code[c] for s in seqs for c in s.upper()]
    offs = [0]
    for s in seqs:
        offs.append(offs[-1] + len(s))
    nbytes = (len(bases) + 3) // 4
    buf = bytearray(max(nbytes, 1))
    for k, v in enumerate(bases):
        buf[k >> 2] |= v << (2 * (k & 3))
    return np.frombuffer(bytes(buf), dtype=np.uint8), np.array(offs, np.int64)


def pack(chars, offsets=None, revcomp: bool = False, nmask: bool = False):
    """Oracle packing of character reads into the 2-bit stream (see the
    header of pack_oracle.c).  chars: uint8 array; offsets: int64 CSR of the
    sequences (needed for revcomp).  Returns (packed uint8 array of
    ceil(n/16)*4 bytes, number of invalid bases), plus the N mask (uint32,
    ceil(n/32) words) when nmask is true (N and n then count as bases)."""
    lib = _load()
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    n = chars.size
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    out = np.zeros(((n + 15) // 16) * 4, np.uint8)
    mask = np.zeros(max((n + 31) // 32, 1), np.uint32) if nmask else None
    bad = lib.oracle_pack_n(_ptr(chars) if n else None, n, _ptr(offsets), offsets.size - 1,
                            1 if revcomp else 0, _ptr(out) if out.size else None,
                            _ptr(mask) if nmask else None)
    if nmask:
        return out, int(bad), mask[: (n + 31) // 32]
    return out, int(bad)


def start_batch(q_seqs, q_offsets, t_seqs, t_offsets, score, q_end, t_end,
                scoring=(1, -4, 6, 1), q_nmask=None, t_nmask=None):
    """Oracle start positions (see the header of start_oracle.c) of the best
    alignments whose score and end are given (the answers of align_batch).
    Returns (q_start, t_start) int64 arrays; raises if an anchored maximum
    differs from the given score."""
    lib = _load()
    n = len(q_offsets) - 1
    arrs = [np.ascontiguousarray(a, dtype=np.int64) for a in (score, q_end, t_end)]
    qs = np.full(n, -1, np.int64)
    ts = np.full(n, -1, np.int64)
    if n == 0:
        return qs, ts
    q_seqs = np.ascontiguousarray(q_seqs, dtype=np.uint8)
    t_seqs = np.ascontiguousarray(t_seqs, dtype=np.uint8)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.int64)
    t_offsets = np.ascontiguousarray(t_offsets, dtype=np.int64)
    a, b, o, e = scoring
    qm = _mask_ptr(q_nmask, q_offsets[-1])
    tm = _mask_ptr(t_nmask, t_offsets[-1])
    bad = lib.oracle_start_batch_n(_ptr(q_seqs), qm[0], _ptr(q_offsets), _ptr(t_seqs), tm[0],
                                   _ptr(t_offsets), n, a, b, o, e, _ptr(arrs[0]),
                                   _ptr(arrs[1]), _ptr(arrs[2]), _ptr(qs), _ptr(ts))
    if bad != 0:
        raise RuntimeError("start oracle: %d pairs whose anchored maximum is not the score" % bad)
    return qs, ts


def align_banded(q_seqs, q_offsets, t_seqs, t_offsets, band: int, scoring=(1, -4, 6, 1),
                 threads: int | None = None):
    """Oracle of Eq. 1 restricted to the band |i - j| <= band (see the header
    of band_oracle.c).  Returns (score, q_end, t_end) int64 arrays."""
    if band < 0:
        raise ValueError("band must be >= 0")
    lib = _load()
    n = len(q_offsets) - 1
    out = [np.zeros(max(n, 0), np.int64) for _ in range(3)]
    if n <= 0:
        return tuple(out)
    q_seqs = np.ascontiguousarray(q_seqs, dtype=np.uint8)
    t_seqs = np.ascontiguousarray(t_seqs, dtype=np.uint8)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.int64)
    t_offsets = np.ascontiguousarray(t_offsets, dtype=np.int64)
    qb = q_seqs if len(q_seqs) else np.zeros(1, np.uint8)
    tb = t_seqs if len(t_seqs) else np.zeros(1, np.uint8)
    a, b, o, e = (int(x) for x in scoring)
    # independent pairs: contiguous ranges on worker threads (ctypes
    # releases the GIL for the call)
    workers = max(1, min(threads or os.cpu_count() or 1, n))
    cuts = np.linspace(0, n, workers + 1).astype(np.int64)

    def run(k):
        lo, hi = int(cuts[k]), int(cuts[k + 1])
        if hi <= lo:
            return 0
        return lib.oracle_align_banded(_ptr(qb), _ptr(q_offsets) + 8 * lo, _ptr(tb),
                                       _ptr(t_offsets) + 8 * lo, hi - lo, a, b, o, e, int(band),
                                       *(_ptr(x) + 8 * lo for x in out))
    if workers == 1:
        rcs = [run(0)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            rcs = list(ex.map(run, range(workers)))
    if any(rc != 0 for rc in rcs):
        raise MemoryError("oracle_align_banded failed")
    return tuple(out)


CIGAR_OPS = {7: "=", 8: "X", 1: "I", 2: "D"}


def cigar_capacity(q_offsets, t_offsets) -> np.ndarray:
    """Offsets of a CIGAR buffer with room for m + n runs per pair (a path
    between start and end has at most m' + n' - 1 runs)."""
    cap = np.diff(np.asarray(q_offsets, np.int64)) + np.diff(np.asarray(t_offsets, np.int64))
    off = np.zeros(len(cap) + 1, np.int64)
    np.cumsum(cap, out=off[1:])
    return off


def trace_batch(q_seqs, q_offsets, t_seqs, t_offsets, score, q_start, q_end, t_start, t_end,
                scoring=(1, -4, 6, 1), cig_off=None, threads: int | None = None):
    """Oracle of the trace (see the header of trace_oracle.c): per pair the
    optimal alignment from (q_start, t_start) to (q_end, t_end) as BAM-coded
    CIGAR runs.  Returns (cig_off, cig, cig_len); cig_len is 0 for score 0
    and -1 for an inconsistent pair (raises RuntimeError if any)."""
    lib = _load()
    n = len(q_offsets) - 1
    if cig_off is None:
        cig_off = cigar_capacity(q_offsets, t_offsets)
    cig_off = np.ascontiguousarray(cig_off, dtype=np.int64)
    cig = np.zeros(max(int(cig_off[-1]) if n > 0 else 0, 1), np.uint32)
    cig_len = np.zeros(max(n, 0), np.int64)
    if n <= 0:
        return cig_off, cig, cig_len
    arr = [np.ascontiguousarray(x, dtype=np.int64) for x in (score, q_start, q_end, t_start, t_end)]
    q_seqs = np.ascontiguousarray(q_seqs, dtype=np.uint8)
    t_seqs = np.ascontiguousarray(t_seqs, dtype=np.uint8)
    qb = q_seqs if len(q_seqs) else np.zeros(1, np.uint8)
    tb = t_seqs if len(t_seqs) else np.zeros(1, np.uint8)
    q_offsets = np.ascontiguousarray(q_offsets, dtype=np.int64)
    t_offsets = np.ascontiguousarray(t_offsets, dtype=np.int64)
    a, b, o, e = (int(x) for x in scoring)
    # independent pairs: contiguous ranges on worker threads (cig_off holds
    # absolute positions, so every range writes into the same cig)
    workers = max(1, min(threads or 1, n))
    cuts = np.linspace(0, n, workers + 1).astype(np.int64)

    def run(k):
        lo, hi = int(cuts[k]), int(cuts[k + 1])
        if hi <= lo:
            return 0
        return lib.oracle_trace_batch(_ptr(qb), _ptr(q_offsets) + 8 * lo, _ptr(tb),
                                      _ptr(t_offsets) + 8 * lo, hi - lo, a, b, o, e,
                                      *(_ptr(x) + 8 * lo for x in arr),
                                      _ptr(cig_off) + 8 * lo, _ptr(cig), _ptr(cig_len) + 8 * lo)
    if workers == 1:
        rcs = [run(0)]
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            rcs = list(ex.map(run, range(workers)))
    if any(rc < 0 for rc in rcs):
        raise MemoryError("oracle_trace_batch failed")
    bad = sum(rcs)
    if bad > 0:
        raise RuntimeError("trace oracle: %d inconsistent pairs" % bad)
    return cig_off, cig, cig_len


def cigar_string(cig, start, length) -> str:
    """Text form of the runs cig[start : start + length]."""
    return "".join("%d%s" % (int(c) >> 4, CIGAR_OPS[int(c) & 15])
                   for c in cig[start:start + length])
