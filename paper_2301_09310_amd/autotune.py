"""Autotuner of the persistent mode's tile shape per length bin: the
lane-group width W and the query columns per lane K.

For every bin of the table (a query-length range, 16-bit or 32-bit cells)
it draws a synthetic batch whose queries fall in that range (targets 1.0 to
1.5 times the query, half of the pairs related), times the persistent
kernel with each admissible (W, K) forced, checks that every shape gives
the same answers, and keeps the fastest.  W is the paper's subwarp-size
knob (SALoBa, Section IV-C, and its sweep of Section V-D): narrow groups
waste less of the wavefront's ramp, wide groups finish a long pair sooner.
K sets the chunk width W*K with W: the padding of a pair's last chunk, how
often the boundary column is handed over, and the registers per lane
(K = 32 runs 2 waves per SIMD instead of 3).

The per-bin sweep sees each bin alone.  In a real batch every column class
is its own persistent launch, and 32 columns per lane run two waves per SIMD
instead of three, so a second phase confirms each non-default column count
on whole workloads: starting from every bin at its best width for 16
columns, it switches one bin at a time to its sweep-best (W, K) and keeps
the switch only if the reference workloads (a 400,000-pair slice of the
mixed batch and 1,000,000 short reads) get at least 0.5% faster in total.

Usage (on the GPU):
  python -m paper_2301_09310_amd.autotune --out paper_2301_09310_amd/tune_gfx950.json
The JSON holds the table and every measurement.  The library's build
(paper_2301_09310_amd/build.py) compiles the JSON's table in as the
built-in default, and salo.load_tune_table(path) installs another record at
run time.
"""
from __future__ import annotations

import argparse
import datetime
import json
import os
import sys
import time

import numpy as np

WIDTHS = (1, 2, 4, 8, 16, 32, 64)
COLS = (8, 16, 32)
ROWS_PER_LANE = 1024     # a width-W bin admits targets of up to 1024*W bases


def bin_batch(m_lo: int, m_hi: int, cells: float, seed: int, min_pairs: int = 256):
    """Pairs with queries in (m_lo, m_hi], targets 1.0-1.5x, ~`cells` cells."""
    from paper_2301_09310_amd import inputs as I
    rng = np.random.default_rng([seed, m_hi])
    lo = max(m_lo + 1, 1)
    hi = min(m_hi, 12000)
    mean_cells = ((lo + hi) / 2.0) ** 2 * 1.25
    # enough pairs for the target cell count, and for several units per
    # resident wave even at the widest width (2 pairs per unit)
    n = int(max(min_pairs, min(2_000_000, cells / mean_cells)))
    ql = rng.integers(lo, hi + 1, n)
    tl = np.minimum(np.rint(ql * rng.uniform(1.0, 1.5, n)).astype(np.int64), 65535)
    qs, ts = [], []
    t_all = rng.integers(0, 4, int(tl.sum()), dtype=np.uint8)
    q_all = rng.integers(0, 4, int(ql.sum()), dtype=np.uint8)
    to = np.concatenate([[0], np.cumsum(tl)])
    qo = np.concatenate([[0], np.cumsum(ql)])
    related = rng.random(n) < 0.5
    for p in np.nonzero(related)[0]:
        # copy a window of the target into the query (with no mutations: the
        # width choice depends on shape, not on the alignment's content)
        k = int(min(ql[p], tl[p]))
        q_all[qo[p]:qo[p] + k] = t_all[to[p]:to[p] + k]
    b = I.Batch(I.pack_bases(q_all), qo.astype(np.int64), I.pack_bases(t_all),
                to.astype(np.int64))
    return b


def time_config(dev_batch, n, reps=3, **opts):
    import torch
    from paper_2301_09310_amd import salo
    q, qo, t, to = dev_batch
    out = tuple(torch.empty(n, dtype=torch.int32, device=q.device) for _ in range(3))
    salo.align_batch(q, qo, t, to, out=out, **opts)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        salo.align_batch(q, qo, t, to, out=out, timing=True, **opts)
        ms.append(sum(salo.last_timing()))
    return float(np.median(ms)), out


def tune(cells_per_bin: float = 2e10, cols=COLS, seed: int = 7, log=print):
    import torch
    from paper_2301_09310_amd import salo
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    min_pairs = 4 * cus * 12 * 2      # 4 units per resident wave at 2 pairs/unit
    salo.set_bins(None)
    table = salo.get_bins()
    prev = {0: 0, 1: 0}
    result = []
    for m_hi, packed, _w, _k in table:
        m_lo = prev[packed]
        prev[packed] = m_hi
        b = bin_batch(m_lo, m_hi, cells_per_bin, seed, min_pairs=min_pairs)
        n_max = int(b.t_lens().max())
        dev = salo.to_device(b)
        timings = {}
        ref = None
        for k in cols:
            for w in WIDTHS:
                if n_max > ROWS_PER_LANE * w:
                    continue
                ms, out = time_config(dev, b.n_pairs, mode="persistent", lanes=w, cols=k,
                                      force_int32=not packed)
                res = tuple(x.cpu() for x in out)
                if ref is None:
                    ref = res
                elif not all(torch.equal(x, y) for x, y in zip(res, ref)):
                    raise RuntimeError("lanes %d cols %d changed the results of bin %d"
                                       % (w, k, m_hi))
                timings[(w, k)] = ms
        best = min(timings, key=timings.get)
        gcups = b.cells() / (timings[best] * 1e-3) / 1e9
        log("bin m<=%5d %s: %d pairs %.2e cells; best lanes %d cols %d (%.0f GCUPS); %s" % (
            m_hi, "16-bit" if packed else "32-bit", b.n_pairs, b.cells(), best[0], best[1],
            gcups, " ".join("%dx%d:%.2fms" % (w, k, t) for (w, k), t in timings.items())))
        result.append({"m_hi": m_hi, "packed": packed, "lanes": best[0], "cols": best[1],
                       "pairs": b.n_pairs, "cells": b.cells(),
                       "ms": {"%dx%d" % wk: round(t, 4) for wk, t in timings.items()}})
    return result


def confirm(bins, seed: int = 0, reps: int = 3, log=print):
    """Phase two: bins whose sweep-best K is not 16 keep it only if the
    reference workloads get faster with it (see the module docstring)."""
    import torch
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo
    refs = [salo.to_device(I.mixed(seed, 400_000)), salo.to_device(I.short_reads(seed, 1_000_000))]

    def total(table):
        salo.set_bins([(b["m_hi"], b["packed"], b["lanes"], b["cols"]) for b in table])
        t = 0.0
        for d in refs:
            n = d[1].numel() - 1
            t += time_config(d, n, reps=reps)[0]
        return t

    base = []
    for b in bins:
        k16 = {wk: t for wk, t in b["ms"].items() if wk.endswith("x16")}
        w16 = min(k16, key=k16.get) if k16 else "%dx16" % b["lanes"]
        base.append(dict(b, lanes=int(w16.split("x")[0]), cols=16))
    cur = total(base)
    log("phase 2: all bins at 16 columns: %.2f ms on the reference workloads" % cur)
    trials = []
    for i, b in enumerate(bins):
        if b["cols"] == 16:
            continue
        trial = [dict(x) for x in base]
        trial[i] = dict(trial[i], lanes=b["lanes"], cols=b["cols"])
        t = total(trial)
        keep = t < cur * 0.995
        log("phase 2: bin m<=%d %s at %dx%d: %.2f ms (%s)" % (
            b["m_hi"], "16-bit" if b["packed"] else "32-bit", b["lanes"], b["cols"], t,
            "kept" if keep else "not kept"))
        trials.append({"m_hi": b["m_hi"], "packed": b["packed"], "lanes": b["lanes"],
                       "cols": b["cols"], "ms": round(t, 3), "base_ms": round(cur, 3),
                       "kept": keep})
        if keep:
            base, cur = trial, t
    salo.set_bins(None)
    for b, s in zip(bins, base):
        b["sweep_best"] = "%dx%d" % (b["lanes"], b["cols"])
        b["lanes"], b["cols"] = s["lanes"], s["cols"]
    return trials


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "tune_gfx950.json"))
    ap.add_argument("--cells-per-bin", type=float, default=2e10)
    ap.add_argument("--cols", default="8,16,32", help="column counts to try")
    args = ap.parse_args(argv)
    cols = tuple(int(x) for x in args.cols.split(","))
    import torch
    from paper_2301_09310_amd import salo
    salo.load()
    t0 = time.time()
    say = lambda *a: print(*a, flush=True)
    bins = tune(args.cells_per_bin, cols, log=say)
    trials = confirm(bins, log=say)
    props = torch.cuda.get_device_properties(0)
    rec = {"arch": getattr(props, "gcnArchName", "gfx950"), "device": props.name,
           "cus": props.multi_processor_count, "cols_tried": list(cols),
           "date": datetime.date.today().isoformat(), "seconds": round(time.time() - t0, 1),
           "bins": bins, "phase2": trials}
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", args.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
