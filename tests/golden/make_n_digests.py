#!/usr/bin/env python3
"""Write tests/golden/n_digests.json: the oracle's answers for EVERY pair of
the short-read workload with 1% of the bases of both streams marked N, as
sha256 digests.

This script calls only the CPU oracle (oracle/) and the seeded input
generators (paper_2301_09310_amd/inputs.py: the batch, and the N masks of
random_n_masks, which hold no alignment arithmetic).  Nothing here runs or
reads the GPU path.

What is stored for short_reads (2,000,000 pairs, seed 0, scoring
(1, -4, 6, 1)) with N masks of fraction 0.01 (seed 0): the dataset sha256,
the sha256 of each mask, the sha256 of the int32 score, q_end and t_end
arrays, the same per 65,536-pair chunk, and plain sums, as
make_full_digests.py stores for the batches without N.  An N scores a
mismatch against every base, N included (Section II-B names the fifth
letter; the paper gives it no score).  About a minute on eight cores.

Usage: python tests/golden/make_n_digests.py [--threads N]
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
sys.path.insert(0, HERE)

from oracle import oracle as O                      # noqa: E402
from paper_2301_09310_amd import inputs as I        # noqa: E402
from make_full_digests import chunk_digests, digest, CHUNK   # noqa: E402

OUT = os.path.join(HERE, "n_digests.json")
SCORING = (1, -4, 6, 1)
FRACTION = 0.01


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=O.default_threads())
    args = ap.parse_args(argv)
    t0 = time.time()
    b = I.short_reads(0)
    qm, tm = I.random_n_masks(int(b.q_offsets[-1]), int(b.t_offsets[-1]), FRACTION, 0)
    print("short_reads with N: %d pairs generated in %.1fs" % (b.n_pairs, time.time() - t0),
          flush=True)
    t1 = time.time()
    s, qe, te = (x.astype(np.int32) for x in O.align_batch(
        b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, SCORING, nthreads=args.threads,
        q_nmask=qm, t_nmask=tm))
    dt = time.time() - t1
    print("oracle %.1fs" % dt, flush=True)
    mask_sha = lambda m: hashlib.sha256(np.ascontiguousarray(m, "<u4").tobytes()).hexdigest()
    table = {
        "_about": ("Oracle answers (oracle/gotoh_oracle.c, Eq. 1 with N scoring a mismatch) of "
                   "every pair of short_reads with %g of the bases of both streams marked N "
                   "(inputs.random_n_masks, seed 0), scoring %s, as sha256 of little-endian "
                   "int32 arrays; chunks of %d pairs. Written by tests/golden/make_n_digests.py "
                   "(oracle and input generators only)." % (FRACTION, list(SCORING), CHUNK)),
        "short_reads_n001": {
            "generator": I.GENERATOR_VERSION, "seed": 0, "pairs": b.n_pairs,
            "n_fraction": FRACTION, "n_seed": 0, "scoring": list(SCORING),
            "dataset_sha256": b.sha256(), "q_nmask": mask_sha(qm), "t_nmask": mask_sha(tm),
            "score": digest(s), "q_end": digest(qe), "t_end": digest(te),
            "chunk_pairs": CHUNK, "chunks": chunk_digests(s, qe, te),
            "checksums": {"score": int(s.astype(np.int64).sum()),
                          "q_end": int(qe.astype(np.int64).sum()),
                          "t_end": int(te.astype(np.int64).sum()),
                          "zero_scores": int((s == 0).sum())},
            "oracle_seconds": round(dt, 1), "oracle_threads": args.threads,
        },
    }
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)
    print("written %s in %.1fs" % (OUT, time.time() - t0), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
