#!/usr/bin/env python3
"""Write tests/golden/full_digests.json: the oracle's answers for EVERY pair
of the four batch workloads, as sha256 digests.

This script calls only the CPU oracle (oracle/) and the seeded input
generator (paper_2301_09310_amd/inputs.py, which holds no alignment
arithmetic).  Nothing here runs or reads the GPU path.

What is stored, per workload (plain_small 1,000 pairs, short_reads
2,000,000, long_uneven 200,000, mixed 4,000,000; seed 0, scoring
(1, -4, 6, 1)):
  * dataset_sha256 -- Batch.sha256() of the generated batch, so a test can
    tell a changed generator from a changed answer;
  * score / q_end / t_end -- sha256 of each answer array as little-endian
    int32 (Eq. 1 of Section II-A: the maximum H and its first position in
    row-major order over target rows and query columns);
  * chunks -- sha256 of the three arrays of every run of CHUNK consecutive
    pairs (score bytes, then q_end, then t_end), so that a mismatch can be
    narrowed to a few thousand pairs and compared pair by pair;
  * checksums -- plain sums of the three arrays (a second, readable check).

The oracle's work is split into pieces of PIECE pairs whose answers are
cached (by dataset digest and piece) under --cache, so an interrupted run
resumes.  The mixed workload is about 9.8e12 cells: roughly an hour on
eight cores.

Usage: python tests/golden/make_full_digests.py [--only NAME ...]
                                                [--threads N] [--cache DIR]
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

OUT = os.path.join(HERE, "full_digests.json")
SCORING = (1, -4, 6, 1)
CHUNK = 1 << 16          # pairs per chunk digest
PIECE = 1 << 18          # pairs per cached oracle piece (a multiple of CHUNK)
NAMES = ("plain_small", "short_reads", "long_uneven", "mixed")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def chunk_digests(score, qend, tend, chunk=CHUNK):
    """sha256 of (score, q_end, t_end) int32 bytes of each run of `chunk` pairs."""
    out = []
    for c0 in range(0, len(score), chunk):
        h = hashlib.sha256()
        for a in (score, qend, tend):
            h.update(np.ascontiguousarray(a[c0:c0 + chunk], dtype="<i4").tobytes())
        out.append(h.hexdigest())
    return out


def oracle_answers(batch, threads, cache_dir, tag, log):
    """(score, q_end, t_end) int32 of every pair, in pieces of PIECE pairs,
    each cached as an .npz of int32 arrays."""
    n = batch.n_pairs
    parts = []
    for p0 in range(0, n, PIECE):
        p1 = min(n, p0 + PIECE)
        path = os.path.join(cache_dir, "%s_%d_%d.npz" % (tag, p0, p1)) if cache_dir else None
        if path and os.path.exists(path):
            with np.load(path) as z:
                parts.append((z["score"], z["qend"], z["tend"]))
            continue
        sub = batch.subset(np.arange(p0, p1))
        t0 = time.time()
        s, qe, te = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets,
                                  SCORING, nthreads=threads)
        res = tuple(x.astype(np.int32) for x in (s, qe, te))
        if path:
            tmp = path + ".tmp.npz"
            np.savez(tmp, score=res[0], qend=res[1], tend=res[2])
            os.replace(tmp, path)
        parts.append(res)
        log("  pairs %d..%d: %.3e cells in %.1fs" % (p0, p1, sub.cells(), time.time() - t0))
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(3))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--threads", type=int, default=O.default_threads())
    ap.add_argument("--cache", default=os.path.join("/tmp", "salo_digest_cache"))
    args = ap.parse_args(argv)
    names = args.only or list(NAMES)
    os.makedirs(args.cache, exist_ok=True)

    def log(msg):
        print(msg, flush=True)

    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    table["_about"] = (
        "Oracle answers (oracle/gotoh_oracle.c, Eq. 1) of every pair of each workload, "
        "seed 0, scoring %s, as sha256 of little-endian int32 arrays; chunks of %d pairs. "
        "Written by tests/golden/make_full_digests.py (oracle and input generator only)."
        % (list(SCORING), CHUNK))
    for name in names:
        t0 = time.time()
        batch = I.WORKLOADS[name](0)
        ds = batch.sha256()
        log("%s: %d pairs, %.3e cells, generated in %.1fs" % (
            name, batch.n_pairs, batch.cells(), time.time() - t0))
        t1 = time.time()
        s, qe, te = oracle_answers(batch, args.threads, args.cache, ds[:16], log)
        dt = time.time() - t1
        table[name] = {
            "generator": I.GENERATOR_VERSION,
            "seed": 0,
            "pairs": batch.n_pairs,
            "cells": batch.cells(),
            "scoring": list(SCORING),
            "dataset_sha256": ds,
            "score": digest(s),
            "q_end": digest(qe),
            "t_end": digest(te),
            "chunk_pairs": CHUNK,
            "chunks": chunk_digests(s, qe, te),
            "checksums": {"score": int(s.astype(np.int64).sum()),
                          "q_end": int(qe.astype(np.int64).sum()),
                          "t_end": int(te.astype(np.int64).sum()),
                          "zero_scores": int((s == 0).sum())},
            "oracle_seconds": round(dt, 1),
            "oracle_threads": args.threads,
        }
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(tmp, OUT)
        log("%s: oracle %.1fs on %d threads (%.3f GCUPS); digests written" % (
            name, dt, args.threads, batch.cells() / max(dt, 1e-9) / 1e9))
        del batch
    return 0


if __name__ == "__main__":
    sys.exit(main())
