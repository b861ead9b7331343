#!/usr/bin/env python3
"""Throughput benchmark of the batched seed-extension hot path on one GPU.

One step = one salo_align_batch call over the whole synthetic batch (every
pair's affine-gap Smith-Waterman-Gotoh table, Section II-A Eq. 1, plus its
maximum and end position), inputs already resident in HBM.  Prints ONE JSON
line.  The default workload is the short-read extension batch: 2,000,000
pairs, query length U{50..250}, target = source + U{0..100} flank, 1%
substitutions, 0.1% indels, 10% unrelated pairs, scoring (1, -4, 6, 1).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload short_reads|plain_small|long_uneven|mixed]
                       [--mode auto|plain|persistent] [--lanes L --cols C]
                       [--no-cpu-baseline] [--parity-sample N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS (bit-exact vs oracle) on mixed-length batches; p50/p99 latency at fixed rate"
SCORING = (1, -4, 6, 1)
# Algorithmic integer operations per DP cell (Eq. 1): S select (2), diagonal
# add (1), E (2), F (2), H = max of four (2), H - alpha (1), running max (1).
OPS_PER_CELL = 11
# gfx950 VALU: 256 CUs x 64 lanes x 2.4 GHz; packed 16-bit ops do 2 elements.
PEAK_TOPS = {"u16x2": 256 * 64 * 2.4e9 * 2 / 1e12, "i32": 256 * 64 * 2.4e9 / 1e12}
PEAK_TOPS["f16x2"] = PEAK_TOPS["f16x2+u16x2"] = PEAK_TOPS["u16x2"]   # packed 16-bit rate
HBM_PEAK_GBS = 8000.0


def subset_masks(batch, idx, masks):
    """N masks of batch.subset(idx): the sampled pairs' bits, in the
    subset's stream layout."""
    out = []
    for mask, off in zip(masks, (batch.q_offsets, batch.t_offsets)):
        if mask is None:
            out.append(None)
            continue
        bits = np.unpackbits(mask.view(np.uint8), bitorder="little")
        parts = [bits[off[p]:off[p + 1]] for p in idx]
        sel = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        words = np.zeros(max((sel.size + 31) // 32, 1), np.uint32)
        packed = np.packbits(sel, bitorder="little")
        words.view(np.uint8)[: packed.size] = packed
        out.append(words)
    return out


def cell_dtype(batch, scoring=SCORING, n_masks=False) -> str:
    """Cell arithmetic the library picks for this batch: binary16 where a
    pair's best score is at most 2048 (the scoring fits the binary16 row
    table), 16-bit integers elsewhere (32-bit beyond the 16-bit bound)."""
    match, mism = scoring[0], scoring[1]
    mn = np.minimum(batch.q_lens(), batch.t_lens())
    half = (match * mn <= 2048) & (not n_masks)
    u16 = match * (mn + 1) - mism <= 0x7BFF
    if n_masks and u16.all():
        return "u16x2"
    if half.all():
        return "f16x2"
    if (half | u16).all():
        return "f16x2+u16x2"
    return "i32"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(files=("salo_kernels.hip", "salo_internal.h")) -> str:
    """sha256 of a kernel's sources (the DP kernel by default); profiler
    byte counts are only valid for the kernel they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2301_09310_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, source_hash=None):
    """HBM bytes per DP launch for this kernel source and workload, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded in traffic.json (scaled
    by the plain-copy calibration); None when not measured for this source."""
    path = os.path.join(ROOT, "paper_2301_09310_amd", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    rec = table.get(source_hash or kernel_source_hash(), {}).get(workload)
    return None if rec is None else float(rec["bytes_per_launch"])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    help="default short_reads (anchored_long with --band)")
    ap.add_argument("--pairs", type=int, default=0, help="override the pair count")
    ap.add_argument("--mode", default="auto")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--cols", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--parity-sample", type=int, default=3000)
    ap.add_argument("--compare-plain", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="served stream: Poisson arrivals of 1-4096-pair requests drawn from "
                         "the mixed workload; prints p50/p99 latency at 0.5x/0.8x/1.2x of the "
                         "saturated request rate")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-pool", type=int, default=1_000_000)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-slots", type=int, default=3,
                    help="launches in flight at once (one HIP stream each)")
    ap.add_argument("--serve-launch-pairs", type=int, default=1 << 17,
                    help="most pairs merged into one launch")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step (plan + DP launches) in a HIP graph and time replays")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 3 device-to-device copies of BYTES bytes (a known-"
                         "traffic kernel for scaling the profiler's byte counters)")
    ap.add_argument("--plain-lanes", type=int, default=4)
    ap.add_argument("--n-fraction", type=float, default=0.0,
                    help="mark this fraction of bases (both streams, seeded) as N and "
                         "align through the N-mask entry point")
    ap.add_argument("--starts", action="store_true",
                    help="also time the start-position pass on the timed step's answers")
    ap.add_argument("--band", type=int, default=-1, metavar="W",
                    help="time the banded pass (cells with |i - j| <= W) instead")
    ap.add_argument("--trace", action="store_true",
                    help="time the trace pass (CIGAR of each best alignment) instead")
    ap.add_argument("--trace-workspace-gb", type=float, default=16.0)
    ap.add_argument("--pack", action="store_true",
                    help="time the on-device packing of the workload's reads written as "
                         "characters (forward and reverse-complement)")
    args = ap.parse_args(argv)
    if args.workload is None:
        args.workload = "anchored_long" if args.band >= 0 else "short_reads"

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(pairs are independent; see DESIGN.md for how it would shard)",
              file=sys.stderr)
        return 2

    import torch
    from oracle import oracle as O
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    salo.load()
    dev = torch.device("cuda:0")

    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes 3 times" % args.calibrate_copy)
        return 0

    if args.serve:
        return serve_bench(args)
    if args.pack:
        return pack_bench(args)
    if args.band >= 0:
        return band_bench(args)
    if args.trace:
        return trace_bench(args)

    gen = I.WORKLOADS[args.workload]
    t0 = time.time()
    kw = {}
    if args.workload in ("short_reads", "long_uneven", "mixed"):
        last = [time.time()]

        def progress(done, total):
            if time.time() - last[0] > 10:
                last[0] = time.time()
                log("generating %s: %d / %d pairs" % (args.workload, done, total))
        kw["progress"] = progress
    batch = gen(0, args.pairs, **kw) if args.pairs else gen(0, **kw)
    cells = batch.cells()
    log("workload %s: %d pairs, %.3e cells, generated in %.1fs" % (
        args.workload, batch.n_pairs, cells, time.time() - t0))

    q, qo, t, to = salo.to_device(batch, dev)
    n = batch.n_pairs
    q_nmask = t_nmask = None
    masks_np = (None, None)
    if args.n_fraction > 0:
        rng_n = np.random.default_rng([0, 99])

        def n_mask(total):
            bits = rng_n.random(total) < args.n_fraction
            words = np.zeros(max((total + 31) // 32, 1), np.uint32)
            idx = np.nonzero(bits)[0]
            np.bitwise_or.at(words, idx >> 5, np.uint32(1) << (idx & 31).astype(np.uint32))
            return words
        masks_np = (n_mask(int(batch.q_offsets[-1])), n_mask(int(batch.t_offsets[-1])))
        q_nmask = torch.from_numpy(masks_np[0].view(np.int32)).to(dev)
        t_nmask = torch.from_numpy(masks_np[1].view(np.int32)).to(dev)
    out = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(3))
    opts = dict(mode=args.mode, lanes=args.lanes, cols=args.cols,
                waves_per_cu=args.waves_per_cu)
    if q_nmask is not None:
        opts.update(q_nmask=q_nmask, t_nmask=t_nmask)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
    torch.cuda.synchronize()

    graph = None
    if args.graph:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            salo.reserve(n, stream=stream)
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
        torch.cuda.synchronize()

    # timed region: K steps between events recorded on the launch stream;
    # the library also records events around its plan and DP kernels
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan_ms, dp_ms = [], []
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        if graph is not None:
            with torch.cuda.stream(stream):     # replays run on the current stream
                graph.replay()
            continue
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, timing=True, **opts)
        a, b = salo.last_timing(stream)
        plan_ms.append(a)
        dp_ms.append(b)
    ev1.record(stream)
    if graph is not None:
        # kernel durations of one replayed step, from a separate timed call
        torch.cuda.synchronize()
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, timing=True, **opts)
        a, b = salo.last_timing(stream)
        plan_ms.append(a)
        dp_ms.append(b)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    gcups = cells * args.steps / (total_ms * 1e-3) / 1e9
    log("plan ms: %s" % " ".join("%.3f" % x for x in plan_ms))
    log("dp ms:   %s (wall %.3fs)" % (" ".join("%.2f" % x for x in dp_ms), wall))

    comparison = None
    if args.compare_plain and args.mode != "plain":
        popts = dict(mode="plain", lanes=args.plain_lanes, cols=16,
                     waves_per_cu=args.waves_per_cu)
        if q_nmask is not None:
            popts.update(q_nmask=q_nmask, t_nmask=t_nmask)
        t_first = time.perf_counter()
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **popts)
        torch.cuda.synchronize()
        # a plain step of many seconds reports each step (the host waits
        # between steps, so the timed launches stay back to back only when
        # steps are short)
        pm_progress = time.perf_counter() - t_first > 5.0
        log("plain warm-up step: %.1f s" % (time.perf_counter() - t_first))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.steps):
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **popts)
            if pm_progress:
                torch.cuda.synchronize()
                log("plain step %d done" % k)
        e1.record(stream)
        torch.cuda.synchronize()
        pm = e0.elapsed_time(e1) / args.steps
        comparison = {"plain_gcups": round(cells / (pm * 1e-3) / 1e9, 2),
                      "plain_ms_per_step": round(pm, 4), "plain_lanes": args.plain_lanes,
                      "speedup_vs_plain": round(pm / ms_per_step, 3)}
        log("plain lanes=%d: %.2f ms/step" % (args.plain_lanes, pm))
        # the persistent outputs must be what the parity sample checks
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
        torch.cuda.synchronize()

    starts = None
    if args.starts:
        ans = tuple(x.clone() for x in out)
        sq = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(2))
        for _ in range(max(args.warmup, 1)):
            salo.align_starts(q, qo, t, to, ans, SCORING, out=sq, stream=stream, **opts)
        torch.cuda.synchronize()
        s_plan, s_dp = [], []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            salo.align_starts(q, qo, t, to, ans, SCORING, out=sq, stream=stream, timing=True,
                              **opts)
            pm_, dm_ = salo.last_timing(stream)
            s_plan.append(pm_)
            s_dp.append(dm_)
        e1.record(stream)
        torch.cuda.synchronize()
        s_ms = e0.elapsed_time(e1) / args.steps
        a_np = [x.cpu().numpy().astype(np.int64) for x in ans]
        s_cells = int(((a_np[1] + 1) * (a_np[2] + 1) * (a_np[0] > 0)).sum())
        rng_s = np.random.default_rng(4)
        k_s = min(args.parity_sample, n)
        idx_s = np.sort(rng_s.choice(n, size=k_s, replace=False))
        sub_s = batch.subset(idx_s)
        smq, smt = subset_masks(batch, idx_s, masks_np)
        w_ans = O.align_batch(sub_s.q_seqs, sub_s.q_offsets, sub_s.t_seqs, sub_s.t_offsets,
                              SCORING, q_nmask=smq, t_nmask=smt)
        w_st = O.start_batch(sub_s.q_seqs, sub_s.q_offsets, sub_s.t_seqs, sub_s.t_offsets,
                             *w_ans, scoring=SCORING, q_nmask=smq, t_nmask=smt)
        ok_s = all(np.array_equal(g.cpu().numpy()[idx_s].astype(np.int64), w)
                   for g, w in zip(sq, w_st))
        starts = {"ms_per_step": round(s_ms, 4), "dp_ms": round(float(np.mean(s_dp)), 4),
                  "plan_ms": round(float(np.mean(s_plan)), 4), "cells": s_cells,
                  "gcups": round(s_cells / (s_ms * 1e-3) / 1e9, 2),
                  "parity": "bit-exact on %d sampled pairs" % k_s if ok_s else "MISMATCH"}
        log("start pass: %.3f ms per step (DP %.3f), %.1f GCUPS over the reversed prefixes, %s"
            % (s_ms, starts["dp_ms"], starts["gcups"], starts["parity"]))

    # parity on a sample of pairs (the full-size check lives in the tests)
    rng = np.random.default_rng(1)
    k = min(args.parity_sample, n)
    idx = np.sort(rng.choice(n, size=k, replace=False))
    got = [x.cpu().numpy()[idx].astype(np.int64) for x in out]
    sub = batch.subset(idx)
    sqm, stm = subset_masks(batch, idx, masks_np)
    want = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING,
                         q_nmask=sqm, t_nmask=stm)
    parity_ok = all(np.array_equal(g, w) for g, w in zip(got, want))
    log("parity on %d sampled pairs: %s" % (k, "bit-exact" if parity_ok else "MISMATCH"))

    # roofline of the DP kernel: algorithmic int ops per launch / launch time
    dtype = cell_dtype(batch, n_masks=q_nmask is not None)
    kern_ms = float(np.mean(dp_ms))
    achieved = OPS_PER_CELL * cells / (kern_ms * 1e-3) / 1e12
    peak = PEAK_TOPS[dtype]
    traffic = measured_traffic(args.workload)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel": ("plain_kernel" if args.mode == "plain" else "persistent_kernel"),
            "kernel_ms": round(kern_ms, 4), "ops_per_cell": OPS_PER_CELL,
            "traffic_unit": "bytes per launch", "kernel_source": kernel_source_hash()}

    cpu = None
    if not args.no_cpu_baseline:
        m = min(args.cpu_sample, n)
        sub = batch.subset(np.arange(m))
        cmq, cmt = subset_masks(batch, np.arange(m), masks_np)
        thr = O.default_threads()
        c0 = time.perf_counter()
        O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING,
                      nthreads=thr, q_nmask=cmq, t_nmask=cmt)
        dt = time.perf_counter() - c0
        cpu = {"value": round(sub.cells() / dt / 1e9, 4), "unit": "GCUPS", "cores": thr,
               "kind": "oracle",
               "sample": "first %d pairs of the %s batch (%.3e cells), %.1fs" % (
                   m, args.workload, sub.cells(), dt)}

    rec = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n, "cells": cells,
                   "scoring": list(SCORING), "mode": args.mode, "lanes": args.lanes,
                   "cols": args.cols, "parity": "bit-exact on %d sampled pairs" % k
                   if parity_ok else "MISMATCH on sampled pairs",
                   "plan_ms": round(float(np.mean(plan_ms)), 4), "graph": bool(args.graph),
                   "n_fraction": args.n_fraction,
                   "dp_ms": round(kern_ms, 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "comparison": comparison,
        "starts": starts,
    }
    print(json.dumps(rec), flush=True)
    return 0 if parity_ok and (starts is None or starts["parity"] != "MISMATCH") else 1


def band_bench(args) -> int:
    """GCUPS of salo_align_batch_banded over the cells inside the band
    (|i - j| <= W; Section VII-B) on the anchored long workload, with the
    unbanded pass on the same batch for comparison, parity on sampled pairs
    against the banded oracle, the roofline of the DP kernel over the band's
    cells, and the banded oracle timed on the host."""
    import torch
    from oracle import oracle as O
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo
    dev = torch.device("cuda:0")
    w = args.band
    gen = I.WORKLOADS[args.workload]
    t0 = time.time()
    batch = gen(0, args.pairs) if args.pairs else gen(0)
    n = batch.n_pairs
    rect = batch.cells()
    bcells = int(I.band_cells(batch.q_lens(), batch.t_lens(), w).sum())
    log("workload %s: %d pairs, %.3e cells, %.3e in the band %d, generated in %.1fs" % (
        args.workload, n, rect, bcells, w, time.time() - t0))
    q, qo, t, to = salo.to_device(batch, dev)
    out = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(3))
    opts = dict(lanes=args.lanes, cols=args.cols, waves_per_cu=args.waves_per_cu)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        salo.align_banded(q, qo, t, to, w, SCORING, out=out, stream=stream, **opts)
    torch.cuda.synchronize()
    log("banded warm-up done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan_ms, dp_ms = [], []
    ev0.record(stream)
    for _ in range(args.steps):
        salo.align_banded(q, qo, t, to, w, SCORING, out=out, stream=stream, timing=True,
                          **opts)
        a, b = salo.last_timing(stream)
        plan_ms.append(a)
        dp_ms.append(b)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    gcups = bcells / (ms * 1e-3) / 1e9
    log("banded: %.3f ms per step (DP %s), %.1f GCUPS over band cells"
        % (ms, " ".join("%.2f" % x for x in dp_ms), gcups))
    assert salo.error_count(stream) == 0

    # the unbanded pass on the same batch
    full = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(3))
    salo.align_batch(q, qo, t, to, SCORING, out=full, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        salo.align_batch(q, qo, t, to, SCORING, out=full, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / args.steps
    g_np = [x.cpu().numpy().astype(np.int64) for x in out]
    f_np = [x.cpu().numpy().astype(np.int64) for x in full]
    same = float(np.mean((g_np[0] == f_np[0]) & (g_np[1] == f_np[1]) & (g_np[2] == f_np[2])))
    log("unbanded: %.3f ms per step; banded answer = unbanded answer for %.4f of pairs"
        % (fms, same))

    rng = np.random.default_rng(1)
    k = min(args.parity_sample, n, 300)
    idx = np.sort(rng.choice(n, size=k, replace=False))
    sub = batch.subset(idx)
    want = O.align_banded(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, w, SCORING)
    parity_ok = all(np.array_equal(g[idx], x) for g, x in zip(g_np, want))
    log("parity on %d sampled pairs: %s" % (k, "bit-exact" if parity_ok else "MISMATCH"))

    dtype = cell_dtype(batch)
    kern_ms = float(np.mean(dp_ms))
    achieved = OPS_PER_CELL * bcells / (kern_ms * 1e-3) / 1e12
    peak = PEAK_TOPS[dtype]
    wl = "%s_band%d" % (args.workload, w)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(wl), "kernel": "persistent_kernel (banded)",
            "kernel_ms": round(kern_ms, 4), "ops_per_cell": OPS_PER_CELL,
            "cells": "inside the band", "traffic_unit": "bytes per launch",
            "kernel_source": kernel_source_hash()}

    cpu = None
    if not args.no_cpu_baseline:
        m = min(args.cpu_sample, n, 40000)
        csub = batch.subset(np.arange(m))
        thr = O.default_threads()
        c0 = time.perf_counter()
        O.align_banded(csub.q_seqs, csub.q_offsets, csub.t_seqs, csub.t_offsets, w, SCORING,
                       threads=thr)
        dt = time.perf_counter() - c0
        cb = int(I.band_cells(csub.q_lens(), csub.t_lens(), w).sum())
        cpu = {"value": round(cb / dt / 1e9, 4), "unit": "GCUPS over band cells",
               "cores": thr, "kind": "oracle",
               "sample": "first %d pairs of the %s batch (%.3e band cells; the oracle "
                         "visits all %.3e cells of their tables), %.1fs" % (
                             m, args.workload, cb, csub.cells(), dt)}
        log("cpu oracle: %.3f GCUPS over band cells on %d threads" % (cpu["value"], thr))

    rec = {
        "metric": "GCUPS over the cells inside the band (bit-exact vs oracle), banded pass",
        "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n, "band": w, "band_cells": bcells,
                   "table_cells": rect, "scoring": list(SCORING), "lanes": args.lanes,
                   "cols": args.cols, "dp_ms": round(kern_ms, 4),
                   "plan_ms": round(float(np.mean(plan_ms)), 4),
                   "parity": "bit-exact on %d sampled pairs" % k
                   if parity_ok else "MISMATCH on sampled pairs"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "comparison": {"unbanded_ms_per_step": round(fms, 4),
                       "unbanded_gcups_table_cells": round(rect / (fms * 1e-3) / 1e9, 2),
                       "speedup_vs_unbanded": round(fms / ms, 3),
                       "pairs_with_unbanded_answer": round(same, 4)},
    }
    print(json.dumps(rec), flush=True)
    return 0 if parity_ok else 1


def trace_bench(args) -> int:
    """Time of salo_align_trace on the workload's own answers and starts
    (computed first, untimed), GCUPS over the cells of the spans it refills
    (sum of (q_end - q_start + 1) x (t_end - t_start + 1)), parity of sampled
    CIGARs against the trace oracle, and the oracle timed on the host."""
    import torch
    from oracle import oracle as O
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo
    dev = torch.device("cuda:0")
    gen = I.WORKLOADS[args.workload]
    t0 = time.time()
    batch = gen(0, args.pairs) if args.pairs else gen(0)
    n = batch.n_pairs
    log("workload %s: %d pairs, generated in %.1fs" % (args.workload, n, time.time() - t0))
    q, qo, t, to = salo.to_device(batch, dev)
    stream = torch.cuda.current_stream()
    ans = salo.align_batch(q, qo, t, to, SCORING, stream=stream)
    st = salo.align_starts(q, qo, t, to, ans, SCORING, stream=stream)
    a_np = [x.cpu().numpy().astype(np.int64) for x in ans]
    s_np = [x.cpu().numpy().astype(np.int64) for x in st]
    pos = a_np[0] > 0
    span = int(((a_np[1] - s_np[0] + 1) * (a_np[2] - s_np[1] + 1) * pos).sum())
    ws = torch.empty(int(args.trace_workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    cig_off = salo.cigar_offsets(qo, to)
    opts = dict(lanes=args.lanes, cols=args.cols, waves_per_cu=args.waves_per_cu)
    out = None
    for _ in range(max(args.warmup, 1)):
        out = salo.align_trace(q, qo, t, to, ans, st, SCORING, cig_off=cig_off, workspace=ws,
                               stream=stream, **opts)
    torch.cuda.synchronize()
    log("trace warm-up done; span cells %.3e" % span)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan_ms, dp_ms = [], []
    ev0.record(stream)
    for _ in range(args.steps):
        out = salo.align_trace(q, qo, t, to, ans, st, SCORING, cig_off=cig_off, workspace=ws,
                               stream=stream, timing=True, **opts)
        a, b = salo.last_timing(stream)
        plan_ms.append(a)
        dp_ms.append(b)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    errors = salo.error_count(stream)
    gcups = span / (ms * 1e-3) / 1e9
    log("trace: %.3f ms per step (kernel %s), %.1f GCUPS over span cells, %d errors"
        % (ms, " ".join("%.2f" % x for x in dp_ms), gcups, errors))
    off = out[0].cpu().numpy()
    cig = out[1].cpu().numpy().view(np.uint32)
    ln = out[2].cpu().numpy().astype(np.int64)
    runs = int(ln[ln > 0].sum())

    rng = np.random.default_rng(1)
    k = min(args.parity_sample, n, 2000)
    idx = np.sort(rng.choice(n, size=k, replace=False))
    sub = batch.subset(idx)
    w_ans = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING)
    w_st = O.start_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, *w_ans,
                         scoring=SCORING)
    woff, wcig, wln = O.trace_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets,
                                    w_ans[0], w_st[0], w_ans[1], w_st[1], w_ans[2], SCORING,
                                    threads=O.default_threads())
    parity_ok = errors == 0 and np.array_equal(ln[idx], wln) and all(
        np.array_equal(cig[off[p]:off[p] + ln[p]], wcig[woff[j]:woff[j] + wln[j]])
        for j, p in enumerate(idx))
    log("parity on %d sampled pairs: %s" % (k, "bit-exact" if parity_ok else "MISMATCH"))

    kern_ms = float(np.mean(dp_ms))
    achieved = OPS_PER_CELL * span / (kern_ms * 1e-3) / 1e12
    # 16-bit integer cells where a pair's span admits them (no binary16)
    smn = np.minimum(a_np[1] - s_np[0] + 1, a_np[2] - s_np[1] + 1)[pos]
    u16 = SCORING[0] * (smn + 1) - SCORING[1] <= 0x7BFF
    dtype = "u16x2" if u16.all() else ("u16x2+i32" if u16.any() else "i32")
    peak = PEAK_TOPS["u16x2"] if u16.any() else PEAK_TOPS["i32"]
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "traffic": measured_traffic("trace_" + args.workload),
            "kernel": "persistent_kernel (trace)", "kernel_ms": round(kern_ms, 4),
            "ops_per_cell": OPS_PER_CELL, "cells": "of the start-to-end spans",
            "traffic_unit": "bytes per launch", "kernel_source": kernel_source_hash()}

    cpu = None
    if not args.no_cpu_baseline:
        m = min(args.cpu_sample, n)
        csub = batch.subset(np.arange(m))
        c_ans = O.align_batch(csub.q_seqs, csub.q_offsets, csub.t_seqs, csub.t_offsets, SCORING)
        c_st = O.start_batch(csub.q_seqs, csub.q_offsets, csub.t_seqs, csub.t_offsets, *c_ans,
                             scoring=SCORING)
        thr = O.default_threads()
        c0 = time.perf_counter()
        O.trace_batch(csub.q_seqs, csub.q_offsets, csub.t_seqs, csub.t_offsets, c_ans[0],
                      c_st[0], c_ans[1], c_st[1], c_ans[2], SCORING, threads=thr)
        dt = time.perf_counter() - c0
        cspan = int(((c_ans[1] - c_st[0] + 1) * (c_ans[2] - c_st[1] + 1) * (c_ans[0] > 0)).sum())
        cpu = {"value": round(cspan / dt / 1e9, 4), "unit": "GCUPS over span cells",
               "cores": thr, "kind": "oracle",
               "sample": "first %d pairs of the %s batch (%.3e span cells), %.1fs" % (
                   m, args.workload, cspan, dt)}
        log("cpu trace oracle: %.3f GCUPS on %d threads" % (cpu["value"], thr))

    rec = {
        "metric": "GCUPS over the start-to-end spans (bit-exact CIGAR vs oracle), trace pass",
        "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n, "span_cells": span,
                   "cigar_runs": runs, "scoring": list(SCORING), "lanes": args.lanes,
                   "cols": args.cols, "workspace_gb": args.trace_workspace_gb,
                   "dp_ms": round(kern_ms, 4), "plan_ms": round(float(np.mean(plan_ms)), 4),
                   "parity": "bit-exact on %d sampled pairs" % k
                   if parity_ok else "MISMATCH on sampled pairs"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    return 0 if parity_ok else 1


def pack_bench(args) -> int:
    """GB/s of salo_pack_bases on the workload's reads written as characters
    (query and target streams), forward and reverse-complemented, against
    HBM bandwidth; bit-exact check against the packing oracle."""
    import torch
    from oracle import oracle as O
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo
    gen = I.WORKLOADS[args.workload]
    batch = gen(0, args.pairs) if args.pairs else gen(0)
    letters = np.frombuffer(b"ACGT", np.uint8)
    streams = []
    for packed, off in ((batch.q_seqs, batch.q_offsets), (batch.t_seqs, batch.t_offsets)):
        n = int(off[-1])
        codes = (np.unpackbits(packed[: (n + 3) // 4, None], axis=1, bitorder="little")
                 .reshape(-1, 4, 2) @ np.array([1, 2], np.uint8)).reshape(-1)[:n]
        streams.append((letters[codes], off))
    n_chars = sum(c.size for c, _ in streams)
    n_seqs = sum(o.size - 1 for _, o in streams)
    log("pack workload %s: %d characters in 2 streams" % (args.workload, n_chars))
    dev_streams = [(torch.from_numpy(c).cuda(), torch.from_numpy(o).cuda(),
                    torch.empty(((c.size + 15) // 16) * 4, dtype=torch.uint8, device="cuda"))
                   for c, o in streams]
    stream = torch.cuda.current_stream()
    res = {}
    ok = True
    for rc in (False, True):
        for _ in range(max(args.warmup, 1)):
            for c, o, p in dev_streams:
                salo.pack_bases(c, o, revcomp=rc, out=p, stream=stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            for c, o, p in dev_streams:
                salo.pack_bases(c, o, revcomp=rc, out=p, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        # algorithmic bytes: characters in, packed bases out (+ offsets read
        # by the reverse-complement kernel)
        nbytes = n_chars + sum(p.numel() for _, _, p in dev_streams) + \
            (8 * (n_seqs + 2) if rc else 0)
        gbs = nbytes / (ms * 1e-3) / 1e9
        for (c, o), (_, _, p) in zip(streams, dev_streams):
            want, _ = O.pack(c, o, revcomp=rc)
            ok &= np.array_equal(p.cpu().numpy(), want)
        key = "revcomp" if rc else "forward"
        res[key] = {"ms": round(ms, 4), "gbs": round(gbs, 1), "bytes": nbytes}
        log("pack %s: %.3f ms per pass, %.1f GB/s" % (key, ms, gbs))
    cpu = None
    if not args.no_cpu_baseline:
        c0 = time.perf_counter()
        for c, o in streams:
            O.pack(c, o, revcomp=False)
        dt = time.perf_counter() - c0
        cpu = {"value": round(res["forward"]["bytes"] / dt / 1e9, 3), "unit": "GB/s",
               "cores": 1, "kind": "oracle",
               "sample": "both character streams of the %s batch, forward, %.2fs" % (
                   args.workload, dt)}
    fwd = res["forward"]
    pack_hash = kernel_source_hash(("salo_pack.hip",))
    rec = {"metric": "packing GB/s (characters in + packed bases out, bit-exact vs oracle)",
           "value": fwd["gbs"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": max(args.warmup, 1), "ms_per_step": fwd["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": args.workload + " reads as characters",
                      "characters": n_chars, "sequences": n_seqs,
                      "parity": "bit-exact, full streams" if ok else "MISMATCH"},
           "roofline": {"bound": "hbm", "achieved": fwd["gbs"], "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(fwd["gbs"] / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic("pack_" + args.workload, pack_hash),
                        "traffic_unit": "bytes per pass (both streams)",
                        "algorithmic_bytes": fwd["bytes"], "kernel": "pack_forward",
                        "kernel_source": pack_hash},
           "revcomp": res["revcomp"], "cpu_baseline": cpu}
    print(json.dumps(rec), flush=True)
    return 0 if ok else 1


def serve_bench(args) -> int:
    """p50/p99 request latency of the served stream at fixed offered rates."""
    from oracle import oracle as O
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import serve as S
    t0 = time.time()
    pool = I.mixed(0, args.serve_pool)
    log("serve pool: %d mixed pairs in %.1fs" % (pool.n_pairs, time.time() - t0))
    n = args.serve_warmup + args.serve_requests
    sizes = S.request_sizes(n, 1)
    budget = int(args.serve_budget_gb * (1 << 30))
    ex = S.GpuExecutor(n_slots=args.serve_slots, max_pairs=args.serve_launch_pairs,
                       scoring=SCORING)

    def run(rate):
        arr = np.zeros(n) if rate is None else S.poisson_arrivals(n, rate, 1)
        reqs = S.split_requests(pool, sizes, arr)
        st = S.Server(ex, budget_bytes=budget, progress=log).run(reqs,
                                                                 warmup=args.serve_warmup)
        return reqs, st.summary()

    reqs, sat = run(None)              # all requests at once: saturated rate
    log("saturated: %s" % json.dumps(sat))
    rate_sat = sat["requests_per_s"]
    # parity: a sample of served requests against the oracle
    rng = np.random.default_rng(2)
    ok = True
    for r in rng.choice(reqs[args.serve_warmup:], size=20, replace=False):
        b = r.batch
        want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, SCORING)
        ok &= all(np.array_equal(g.astype(np.int64), w) for g, w in zip(r.result, want))
    runs = {}
    for f in (0.5, 0.8, 1.2):
        _, summ = run(f * rate_sat)
        runs["%.1fx" % f] = {"offered_rps": round(f * rate_sat, 2),
                              "p50_ms": round(summ["p50_ms"], 3),
                              "p99_ms": round(summ["p99_ms"], 3),
                              "gcups": round(summ["gcups"], 1),
                              "launches": summ["launches"],
                              "mean_requests_per_launch":
                                  round(summ["mean_requests_per_launch"], 2),
                              "max_inflight": summ["max_inflight"]}
        log("%.1fx: %s" % (f, json.dumps(runs["%.1fx" % f])))
    rec = {"metric": METRIC, "value": runs["0.8x"]["p99_ms"], "unit": "ms (p99 at 0.8x)",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f16x2+u16x2",
           "config": {"workload": "served mixed requests", "requests": args.serve_requests,
                      "warmup_requests": args.serve_warmup, "pairs_per_request": "U{1..4096}",
                      "pool_pairs": pool.n_pairs, "budget_gb": args.serve_budget_gb,
                      "slots": args.serve_slots, "launch_pairs": args.serve_launch_pairs,
                      "parity": "bit-exact on 20 sampled requests" if ok else "MISMATCH"},
           "saturated": {"requests_per_s": round(rate_sat, 2), "gcups": round(sat["gcups"], 1),
                         "mean_requests_per_launch": round(sat["mean_requests_per_launch"], 2),
                         "p50_ms": round(sat["p50_ms"], 3), "p99_ms": round(sat["p99_ms"], 3)},
           "rates": runs}
    print(json.dumps(rec), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
