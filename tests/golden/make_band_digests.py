#!/usr/bin/env python3
"""Write tests/golden/band_digests.json: the band oracle's answers for EVERY
pair of the anchored long workload at band 100, as sha256 digests.

This script calls only the CPU oracle (oracle/) and the seeded input
generator (paper_2301_09310_amd/inputs.py, which holds no alignment
arithmetic).  Nothing here runs or reads the GPU path.

What is stored for anchored_long (200,000 pairs, seed 0, scoring
(1, -4, 6, 1)) at band 100 (the cells with |i - j| <= 100, Section VII-B):
the dataset sha256, the sha256 of the int32 score, q_end and t_end arrays,
the same per 65,536-pair chunk, and plain sums, as make_full_digests.py
stores for the unbanded answers.  A few minutes on eight cores.

Usage: python tests/golden/make_band_digests.py [--threads N]
"""
from __future__ import annotations

import argparse
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

OUT = os.path.join(HERE, "band_digests.json")
SCORING = (1, -4, 6, 1)
BAND = 100


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=O.default_threads())
    args = ap.parse_args(argv)
    t0 = time.time()
    b = I.anchored_long(0)
    print("anchored_long: %d pairs generated in %.1fs" % (b.n_pairs, time.time() - t0),
          flush=True)
    t1 = time.time()
    s, qe, te = (x.astype(np.int32) for x in O.align_banded(
        b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, BAND, SCORING, threads=args.threads))
    dt = time.time() - t1
    print("band oracle %.1fs" % dt, flush=True)
    table = {
        "_about": ("Band oracle answers (oracle/band_oracle.c, Eq. 1 over |i - j| <= %d) of "
                   "every pair of anchored_long, seed 0, scoring %s, as sha256 of little-endian "
                   "int32 arrays; chunks of %d pairs. Written by "
                   "tests/golden/make_band_digests.py (oracle and input generator only)."
                   % (BAND, list(SCORING), CHUNK)),
        "anchored_long_band100": {
            "generator": I.GENERATOR_VERSION, "seed": 0, "pairs": b.n_pairs, "band": BAND,
            "scoring": list(SCORING), "dataset_sha256": b.sha256(),
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
