#!/usr/bin/env python3
"""Write tests/golden/trace_digests.json: the oracle's start positions and
CIGAR traces for EVERY pair of a batch workload (short_reads by default,
or long_uneven), as sha256 digests.

This script calls only the CPU oracle (oracle/) and the seeded input
generator (paper_2301_09310_amd/inputs.py, which holds no alignment
arithmetic).  Nothing here runs or reads the GPU path.

What is stored per workload (short_reads: 2,000,000 pairs; long_uneven:
200,000; seed 0, scoring (1, -4, 6, 1)):
  * dataset_sha256 -- Batch.sha256() of the generated batch;
  * q_start / t_start -- sha256 of each start array as little-endian int32
    (the latest optimal start of each best alignment, Section II-A);
  * cigar_len -- sha256 of the run counts (int32), 0 for a pair of score 0;
  * cigar_runs -- sha256 of every pair's BAM-coded runs (length << 4 | op,
    little-endian uint32), concatenated in pair order;
  * chunks -- per run of CHUNK consecutive pairs, sha256 of its q_start,
    t_start and cigar_len bytes followed by its runs, so that a mismatch can
    be narrowed to a few thousand pairs;
  * checksums -- plain sums (a second, readable check).

About four minutes on eight cores for short_reads and twenty for
long_uneven (the start oracle runs on ranges of pairs in parallel).

Usage: python tests/golden/make_trace_digests.py [--workload NAME] [--threads N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from paper_2301_09310_amd import inputs as I        # noqa: E402

OUT = os.path.join(HERE, "trace_digests.json")
SCORING = (1, -4, 6, 1)
CHUNK = 1 << 16          # pairs per chunk digest


def packed_runs(off, cig, ln):
    """Every pair's runs cig[off[p] : off[p] + ln[p]], concatenated in pair
    order (pairs with ln <= 0 add none), and the start of each pair's runs
    in that concatenation (length n + 1)."""
    ln = np.maximum(np.asarray(ln, dtype=np.int64), 0)
    off = np.asarray(off, dtype=np.int64)[:len(ln)]
    starts = np.zeros(len(ln) + 1, np.int64)
    np.cumsum(ln, out=starts[1:])
    idx = np.repeat(off - starts[:-1], ln) + np.arange(int(starts[-1]), dtype=np.int64)
    return np.asarray(cig, dtype=np.uint32)[idx], starts


def trace_digests(qs, ts, ln, runs, starts, chunk=CHUNK):
    """The digests stored for one batch (see the module docstring)."""
    def h32(a, dt="<i4"):
        return hashlib.sha256(np.ascontiguousarray(a, dtype=dt).tobytes()).hexdigest()
    chunks = []
    for c0 in range(0, len(ln), chunk):
        c1 = min(len(ln), c0 + chunk)
        h = hashlib.sha256()
        for a in (qs, ts, ln):
            h.update(np.ascontiguousarray(a[c0:c1], dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(runs[starts[c0]:starts[c1]], dtype="<u4").tobytes())
        chunks.append(h.hexdigest())
    return {
        "q_start": h32(qs), "t_start": h32(ts), "cigar_len": h32(ln),
        "cigar_runs": h32(runs, "<u4"), "chunk_pairs": chunk, "chunks": chunks,
        "checksums": {"q_start": int(np.asarray(qs, np.int64).sum()),
                      "t_start": int(np.asarray(ts, np.int64).sum()),
                      "runs": int(len(runs)),
                      "run_bases": int((np.asarray(runs, np.int64) >> 4).sum())},
    }


def starts_in_ranges(b, ans, threads):
    """The start oracle over contiguous ranges of pairs on worker threads
    (each call releases the interpreter lock), in pair order."""
    from concurrent.futures import ThreadPoolExecutor
    cuts = np.linspace(0, b.n_pairs, max(1, threads) * 4 + 1).astype(np.int64)

    def run(k):
        idx = np.arange(cuts[k], cuts[k + 1])
        if idx.size == 0:
            return np.zeros(0, np.int64), np.zeros(0, np.int64)
        sub = b.subset(idx)
        return O.start_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets,
                             *(a[idx] for a in ans), scoring=SCORING)
    with ThreadPoolExecutor(max(1, threads)) as ex:
        parts = list(ex.map(run, range(len(cuts) - 1)))
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(2))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="short_reads", choices=("short_reads", "long_uneven"))
    ap.add_argument("--threads", type=int, default=O.default_threads())
    args = ap.parse_args(argv)
    t0 = time.time()
    b = I.WORKLOADS[args.workload](0)
    print("%s: %d pairs generated in %.1fs" % (args.workload, b.n_pairs, time.time() - t0),
          flush=True)
    secs = {}
    t1 = time.time()
    ans = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, SCORING,
                        nthreads=args.threads)
    secs["answers"] = round(time.time() - t1, 1)
    t1 = time.time()
    st = starts_in_ranges(b, ans, args.threads)
    secs["starts"] = round(time.time() - t1, 1)
    t1 = time.time()
    off, cig, ln = O.trace_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, ans[0], st[0],
                                 ans[1], st[1], ans[2], SCORING, threads=args.threads)
    secs["traces"] = round(time.time() - t1, 1)
    print("oracle seconds: %s" % secs, flush=True)
    runs, starts = packed_runs(off, cig, ln)
    rec = {
        "generator": I.GENERATOR_VERSION, "seed": 0, "pairs": b.n_pairs,
        "scoring": list(SCORING), "dataset_sha256": b.sha256(),
        "oracle_seconds": secs, "oracle_threads": args.threads,
    }
    rec.update(trace_digests(st[0], st[1], ln, runs, starts))
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    table["_about"] = ("Oracle start positions (oracle/start_oracle.c) and CIGAR traces "
                       "(oracle/trace_oracle.c) of every pair of each workload, seed 0, "
                       "scoring %s, as sha256 digests; chunks of %d pairs. Written by "
                       "tests/golden/make_trace_digests.py (oracle and input generator only)."
                       % (list(SCORING), CHUNK))
    table[args.workload] = rec
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)
    print("written %s in %.1fs" % (OUT, time.time() - t0), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
