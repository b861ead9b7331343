#!/usr/bin/env python3
"""Throughput benchmark of the batched seed-extension hot path on one GPU.

One step = one salo_align_batch call over the whole synthetic batch (every
pair's affine-gap Smith-Waterman-Gotoh table, Section II-A Eq. 1, plus its
maximum and end position), inputs already resident in HBM.  Prints ONE JSON
line.  The default workload is the batched mixed workload: 4,000,000 pairs,
60% of queries U{100..300}, 35% U{300..1000}, 5% U{1000..10000}, targets
1.2x the source with the source at a random offset, 2% substitutions, 1%
single-base indels, scoring (1, -4, 6, 1); each step (plan + persistent DP
launches) is replayed from a HIP graph.  The line also carries the plain
one-launch kernel on the same batch, the served stream's p50/p99 latency,
every pair's parity against the oracle's stored digests, the roofline of
the DP kernel against the nominal and the measured VALU peaks, and the CPU
oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload mixed|short_reads|plain_small|long_uneven]
                       [--mode auto|plain|persistent] [--lanes L --cols C]
                       [--no-graph] [--no-compare-plain] [--no-serve]
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


def kernel_source_hash(files=("csrc/salo_kernels.hip", "csrc/salo_internal.h",
                              "csrc/salo_host.cpp", "tune_gfx950.json")) -> str:
    """sha256 of a kernel's sources and of what sets its launch shapes (by
    default the DP kernels, the host library that picks their tiles, and the
    compiled-in tile table); profiler byte counts are only valid for the
    kernel and launch shapes they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        path = os.path.join(ROOT, "paper_2301_09310_amd", f)
        if f.endswith(".json"):
            # a tuning record: only the table the build compiles in counts
            with open(path) as fh:
                bins = json.load(fh)["bins"]
            h.update(json.dumps([[b["m_hi"], b["packed"], b["lanes"], b.get("cols", 0)]
                                 for b in bins]).encode())
        else:
            with open(path, "rb") as fh:
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


_CEILINGS = {}


def ceilings():
    """Measured ceilings of this GPU from the microbenchmark library
    (libsalo_ubench.so): packed 16-bit and 32-bit VALU element-ops/s (T/s)
    and the HBM copy rate (GB/s, bytes read + written); {} when the library
    is missing.  Measured once per process (about a second)."""
    if _CEILINGS or _CEILINGS.get("_done"):
        return _CEILINGS
    import ctypes
    path = os.path.join(ROOT, "paper_2301_09310_amd", "libsalo_ubench.so")
    _CEILINGS["_done"] = True
    if not os.path.exists(path):
        return _CEILINGS
    lib = ctypes.CDLL(path)
    lib.salo_ubench.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.salo_ubench.restype = ctypes.c_int
    for kind, key, work, reps, scale in ((0, "pk16_tops", 4000, 5, 1e12),
                                         (1, "i32_tops", 4000, 5, 1e12),
                                         (2, "copy_gbs", 1 << 31, 10, 1e9)):
        ms, units = ctypes.c_double(0), ctypes.c_double(0)
        rc = lib.salo_ubench(kind, work, reps, ctypes.byref(ms), ctypes.byref(units))
        if rc == 0 and ms.value > 0:
            _CEILINGS[key] = units.value / (ms.value * 1e-3) / scale
    if "i32_tops" in _CEILINGS:
        # one 32-bit VALU op per lane per clock: the sustained clock
        _CEILINGS["clock_ghz"] = _CEILINGS["i32_tops"] * 1e12 / (256 * 64) / 1e9
    log("measured ceilings: %s" % json.dumps({k: round(v, 3) for k, v in _CEILINGS.items()
                                              if k != "_done"}))
    return _CEILINGS


def measured_valu_peak(dtype: str):
    """The measured VALU peak for this cell type (element-ops/s, T/s)."""
    c = ceilings()
    key = "i32_tops" if dtype == "i32" else "pk16_tops"
    return c.get(key)


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def first_pairs_with_cells(batch, target_cells: float) -> int:
    """Smallest prefix of pairs holding at least target_cells cells."""
    c = np.cumsum(batch.q_lens().astype(np.int64) * batch.t_lens())
    return int(min(batch.n_pairs, np.searchsorted(c, target_cells) + 1))


def cpu_baseline(O, batch, workload, masks_np, all_cells: float, one_cells: float,
                 cap_pairs: int):
    """The oracle timed on this host: all cores on a leading sample of the
    batch, one core on a smaller leading sample (GCUPS of each)."""
    out = {"kind": "oracle", "unit": "GCUPS", "cpu_model": cpu_model(),
           "nproc": os.cpu_count(), "affinity_cores": O.default_threads()}
    for label, cells, thr in (("all_cores", all_cells, O.default_threads()),
                              ("one_core", one_cells, 1)):
        m = min(first_pairs_with_cells(batch, cells), cap_pairs)
        idx = np.arange(m)
        sub = batch.subset(idx)
        cmq, cmt = subset_masks(batch, idx, masks_np)
        c0 = time.perf_counter()
        O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING,
                      nthreads=thr, q_nmask=cmq, t_nmask=cmt)
        dt = time.perf_counter() - c0
        out[label] = {"gcups": round(sub.cells() / dt / 1e9, 4), "threads": thr,
                      "pairs": m, "cells": sub.cells(), "seconds": round(dt, 2)}
        log("cpu oracle, %s: %d pairs, %.3e cells, %.1fs, %.3f GCUPS" % (
            label, m, sub.cells(), dt, sub.cells() / dt / 1e9))
    a = out["all_cores"]
    out["value"] = a["gcups"]
    out["cores"] = a["threads"]
    out["sample"] = ("first %d pairs of the %s batch (%.3e cells) on %d threads; one core: "
                     "first %d pairs (%.3e cells)" % (a["pairs"], workload, a["cells"],
                                                      a["threads"], out["one_core"]["pairs"],
                                                      out["one_core"]["cells"]))
    return out


def full_parity(batch, workload, n_pairs_default, got, masks=None, n_fraction=0.0):
    """Digest comparison of every pair's answers with the oracle's answers
    stored in tests/golden/full_digests.json, or, for a batch with N masks,
    tests/golden/n_digests.json (both written by scripts that run only the
    oracle and the generators); None when the batch has none."""
    import hashlib
    sha = lambda a, dt: hashlib.sha256(np.ascontiguousarray(a, dtype=dt).tobytes()).hexdigest()
    name = "n_digests.json" if masks is not None else "full_digests.json"
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path) or batch.n_pairs != n_pairs_default:
        return None
    with open(path) as f:
        table = json.load(f)
    if masks is None:
        rec = table.get(workload)
    else:
        rec = next((r for k, r in table.items() if k.startswith(workload + "_n")
                    and isinstance(r, dict) and r.get("n_fraction") == n_fraction), None)
        if rec is not None and (sha(masks[0], "<u4") != rec["q_nmask"] or
                                sha(masks[1], "<u4") != rec["t_nmask"]):
            return None
    if rec is None or rec.get("dataset_sha256") != batch.sha256():
        return None
    ok = True
    for arr, key in zip(got, ("score", "q_end", "t_end")):
        d = hashlib.sha256(np.ascontiguousarray(arr, dtype="<i4").tobytes()).hexdigest()
        ok &= d == rec[key]
    return ok


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None,
                    help="default mixed (anchored_long with --band, short_reads with "
                         "--trace)")
    ap.add_argument("--pairs", type=int, default=0, help="override the pair count")
    ap.add_argument("--mode", default="auto")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--cols", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cells", type=float, default=1.2e11,
                    help="cells of the all-core oracle sample (leading pairs)")
    ap.add_argument("--cpu-one-core-cells", type=float, default=4e9,
                    help="cells of the one-core oracle sample (leading pairs)")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="most pairs in either oracle sample")
    ap.add_argument("--parity-sample", type=int, default=3000)
    ap.add_argument("--no-compare-plain", action="store_true",
                    help="skip the plain-kernel comparison (on by default)")
    ap.add_argument("--compare-plain", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--plain-lanes", type=int, default=64,
                    help="lanes per group of the plain kernel (64: its best width on mixed "
                         "lengths)")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="timed plain steps (a plain step on the mixed batch takes seconds)")
    ap.add_argument("--serve", action="store_true",
                    help="only the served stream: Poisson arrivals of 1-4096-pair requests "
                         "drawn from the mixed workload; p50/p99 latency at 0.5x/0.8x/1.2x of "
                         "the saturated request rate")
    ap.add_argument("--no-serve", action="store_true",
                    help="leave the served-stream block out of the mixed-workload line")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-pool", type=int, default=4_000_000,
                    help="pairs of the mixed workload the requests are carved from")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-slots", type=int, default=3,
                    help="launches in flight at once (one HIP stream each)")
    ap.add_argument("--serve-launch-pairs", type=int, default=1 << 17,
                    help="most pairs merged into one launch")
    ap.add_argument("--serve-rates", default="0.5,0.8",
                    help="offered loads as fractions of the saturated rate")
    ap.add_argument("--serve-split", type=int, default=0,
                    help="split_waves of the served launches (0: off; 4: long pairs on four "
                         "waves each in launches with at most 1024 of them)")
    ap.add_argument("--serve-per-launch", action="store_true",
                    help="complete requests when their whole merged launch ends (no "
                         "per-request counters)")
    ap.add_argument("--graph", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls instead of replays of one captured step (plan + "
                         "DP launches in a HIP graph, the default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 3 device-to-device copies of BYTES bytes (a known-"
                         "traffic kernel for scaling the profiler's byte counters)")
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
        args.workload = ("anchored_long" if args.band >= 0 else
                         "short_reads" if (args.trace or args.pack) else "mixed")
    use_graph = not args.no_graph
    compare_plain = not args.no_compare_plain and args.mode != "plain"

    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (pairs are "
              "independent: a batch would shard as contiguous pair ranges of equal cells, "
              "one process per GPU, with no exchange during compute)", file=sys.stderr)
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
    default_pairs = gen.__defaults__[1] if gen.__defaults__ else None
    cells = batch.cells()
    log("workload %s: %d pairs, %.3e cells, generated in %.1fs" % (
        args.workload, batch.n_pairs, cells, time.time() - t0))

    q, qo, t, to = salo.to_device(batch, dev)
    n = batch.n_pairs
    q_nmask = t_nmask = None
    masks_np = (None, None)
    if args.n_fraction > 0:
        masks_np = I.random_n_masks(int(batch.q_offsets[-1]), int(batch.t_offsets[-1]),
                                    args.n_fraction, 0)
        q_nmask = torch.from_numpy(masks_np[0].view(np.int32)).to(dev)
        t_nmask = torch.from_numpy(masks_np[1].view(np.int32)).to(dev)
    out = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(3))
    opts = dict(mode=args.mode, lanes=args.lanes, cols=args.cols,
                waves_per_cu=args.waves_per_cu)
    if q_nmask is not None:
        opts.update(q_nmask=q_nmask, t_nmask=t_nmask)
    stream = torch.cuda.Stream() if use_graph else torch.cuda.current_stream()

    log("warm-up: %d steps" % args.warmup)
    for _ in range(args.warmup):
        salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
    torch.cuda.synchronize()

    graph = None
    if use_graph:
        with torch.cuda.stream(stream):
            salo.reserve(n, stream=stream)
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, **opts)
        torch.cuda.synchronize()
        log("captured one step (plan + DP launches) in a HIP graph")

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
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    gcups = cells * args.steps / (total_ms * 1e-3) / 1e9
    log("timed %d steps: %.2f ms per step, %.1f GCUPS (wall %.3fs)" % (
        args.steps, ms_per_step, gcups, wall))
    if graph is not None:
        # kernel durations of the replayed step's launches, from timed
        # eager calls of the same step on the same stream
        for _ in range(3):
            salo.align_batch(q, qo, t, to, SCORING, out=out, stream=stream, timing=True,
                             **opts)
            a, b = salo.last_timing(stream)
            plan_ms.append(a)
            dp_ms.append(b)
        torch.cuda.synchronize()
    log("plan ms: %s" % " ".join("%.3f" % x for x in plan_ms))
    log("dp ms:   %s" % " ".join("%.2f" % x for x in dp_ms))

    # every pair's answers against the oracle's stored digests
    got_all = [x.cpu().numpy() for x in out]
    full_ok = full_parity(batch, args.workload, default_pairs, got_all,
                          masks_np if q_nmask is not None else None, args.n_fraction)
    if full_ok is not None:
        log("every pair vs the oracle's digests: %s" % ("bit-exact" if full_ok else "MISMATCH"))

    comparison = None
    if compare_plain:
        popts = dict(mode="plain", lanes=args.plain_lanes, cols=16,
                     waves_per_cu=args.waves_per_cu)
        if q_nmask is not None:
            popts.update(q_nmask=q_nmask, t_nmask=t_nmask)
        pout = tuple(torch.empty(n, dtype=torch.int32, device=dev) for _ in range(3))
        t_first = time.perf_counter()
        salo.align_batch(q, qo, t, to, SCORING, out=pout, stream=stream, **popts)
        torch.cuda.synchronize()
        log("plain warm-up step (lanes %d): %.2f s" % (args.plain_lanes,
                                                      time.perf_counter() - t_first))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(args.plain_steps):
            salo.align_batch(q, qo, t, to, SCORING, out=pout, stream=stream, **popts)
            e1.record(stream)
            torch.cuda.synchronize()           # a plain step takes seconds: report each
            log("plain step %d done" % k)
        pm = e0.elapsed_time(e1) / args.plain_steps
        same = all(torch.equal(a, b) for a, b in zip(out, pout))
        comparison = {"plain_gcups": round(cells / (pm * 1e-3) / 1e9, 2),
                      "plain_ms_per_step": round(pm, 4), "plain_lanes": args.plain_lanes,
                      "plain_cols": 16, "plain_steps": args.plain_steps,
                      "speedup_vs_plain": round(pm / ms_per_step, 3),
                      "plain_answers_equal": bool(same)}
        log("plain lanes=%d: %.2f ms/step; answers equal to the persistent ones: %s" % (
            args.plain_lanes, pm, same))
        del pout

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

    # parity on a sample of pairs, recomputed by the oracle here
    rng = np.random.default_rng(1)
    k = min(args.parity_sample, n)
    idx = np.sort(rng.choice(n, size=k, replace=False))
    got = [x[idx].astype(np.int64) for x in got_all]
    sub = batch.subset(idx)
    sqm, stm = subset_masks(batch, idx, masks_np)
    want = O.align_batch(sub.q_seqs, sub.q_offsets, sub.t_seqs, sub.t_offsets, SCORING,
                         q_nmask=sqm, t_nmask=stm)
    sample_ok = all(np.array_equal(g, w) for g, w in zip(got, want))
    log("parity on %d sampled pairs: %s" % (k, "bit-exact" if sample_ok else "MISMATCH"))
    parity_ok = sample_ok and full_ok is not False
    if full_ok is not None:
        parity = ("bit-exact on all %d pairs (oracle digests) and on %d pairs recomputed by "
                  "the oracle here" % (n, k)) if parity_ok else "MISMATCH"
    else:
        parity = "bit-exact on %d sampled pairs" % k if parity_ok else \
            "MISMATCH on sampled pairs"

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
    measured_peak = measured_valu_peak(dtype)
    if measured_peak is not None:
        roof["measured_peak"] = round(measured_peak, 3)
        roof["frac_of_measured_peak"] = round(achieved / measured_peak, 4)
        roof["measured_ceilings"] = {k: round(v, 3) for k, v in ceilings().items()
                                     if k != "_done"}
    if traffic is not None:
        roof["hbm_frac"] = round(traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)

    serve = None
    if args.workload == "mixed" and not args.no_serve and q_nmask is None:
        del q, qo, t, to
        torch.cuda.empty_cache()
        serve = serve_in_child(args, batch.n_pairs)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(O, batch, args.workload, masks_np, args.cpu_cells,
                           args.cpu_one_core_cells, args.cpu_sample)

    rec = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n, "cells": cells,
                   "scoring": list(SCORING), "mode": args.mode, "lanes": args.lanes,
                   "cols": args.cols, "parity": parity,
                   "plan_ms": round(float(np.mean(plan_ms)), 4), "graph": graph is not None,
                   "n_fraction": args.n_fraction,
                   "dp_ms": round(kern_ms, 4)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "comparison": comparison,
        "serve": serve,
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
    pack_hash = kernel_source_hash(("csrc/salo_pack.hip",))
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


def serve_block(args, pool):
    """Served stream on the GPU: Poisson arrivals of requests of U{1..4096}
    pairs carved from consecutive pairs of `pool` (a mixed batch), served by
    continuous batching with admission by HBM footprint.  Runs all requests
    at once to find the saturated rate, then open-loop Poisson streams at the
    fractions of it given by --serve-rates; returns p50/p99 latency and
    GCUPS per rate, with the served answers of sampled requests checked
    against the oracle."""
    from oracle import oracle as O
    from paper_2301_09310_amd import serve as S
    n = args.serve_warmup + args.serve_requests
    sizes = S.request_sizes(n, 1)
    budget = int(args.serve_budget_gb * (1 << 30))
    t0 = time.time()
    base = S.split_requests(pool, sizes, np.zeros(n))
    log("serve: %d requests (%d pairs) carved from the %d-pair pool in %.1fs" % (
        n, int(sizes.sum()), pool.n_pairs, time.time() - t0))
    ex = S.GpuExecutor(n_slots=args.serve_slots, max_pairs=args.serve_launch_pairs,
                       scoring=SCORING, per_request=not args.serve_per_launch,
                       split_waves=args.serve_split)

    def run(rate):
        arr = np.zeros(n) if rate is None else S.poisson_arrivals(n, rate, 1)
        reqs = S.with_arrivals(base, arr)
        k0 = len(ex.launch_split)
        st = S.Server(ex, budget_bytes=budget, progress=log).run(reqs,
                                                                 warmup=args.serve_warmup)
        summ = st.summary()
        ls = ex.launch_split[k0:]
        summ["split_launches"] = sum(1 for x in ls if x > 1)
        return reqs, summ

    reqs, sat = run(None)              # all requests at once: saturated rate
    log("serve saturated: %s" % json.dumps(sat))
    rate_sat = sat["requests_per_s"]
    rng = np.random.default_rng(2)
    ok = True
    checked = rng.choice(np.arange(args.serve_warmup, n), size=min(20, args.serve_requests),
                         replace=False)
    runs = {}
    for f in [float(x) for x in args.serve_rates.split(",") if x]:
        reqs, summ = run(f * rate_sat)
        for k in checked:
            b = reqs[k].batch
            want = O.align_batch(b.q_seqs, b.q_offsets, b.t_seqs, b.t_offsets, SCORING)
            ok &= reqs[k].status == "done" and all(
                np.array_equal(g.astype(np.int64), w) for g, w in zip(reqs[k].result, want))
        runs["%.1fx" % f] = {"offered_rps": round(f * rate_sat, 2),
                              "p50_ms": round(summ["p50_ms"], 3),
                              "p99_ms": round(summ["p99_ms"], 3),
                              "gcups": round(summ["gcups"], 1),
                              "launches": summ["launches"],
                              "mean_requests_per_launch":
                                  round(summ["mean_requests_per_launch"], 2),
                              "max_inflight": summ["max_inflight"],
                              "split_launches": summ["split_launches"]}
        log("serve %.1fx: %s" % (f, json.dumps(runs["%.1fx" % f])))
    return {"requests": args.serve_requests, "warmup_requests": args.serve_warmup,
            "completion": "per launch" if args.serve_per_launch else "per request",
            "split_waves": args.serve_split,
            "split_rule": ("launches with at most 1024 queries above 1024 bases"
                           if args.serve_split > 1 else None),
            "pairs_per_request": "U{1..4096}", "arrivals": "Poisson (seed 1)",
            "budget_gb": args.serve_budget_gb, "slots": args.serve_slots,
            "launch_pairs": args.serve_launch_pairs,
            "parity": ("bit-exact on %d sampled requests at every rate" % len(checked))
            if ok else "MISMATCH",
            "saturated": {"requests_per_s": round(rate_sat, 2), "gcups": round(sat["gcups"], 1),
                          "mean_requests_per_launch": round(sat["mean_requests_per_launch"], 2),
                          "p50_ms": round(sat["p50_ms"], 3), "p99_ms": round(sat["p99_ms"], 3)},
            "rates": runs}


def serve_in_child(args, pool_pairs: int):
    """The served stream of the mixed-workload line, measured by `bench.py
    --serve` in a process of its own (a server's process: its HIP context and
    hardware queues hold only the server's streams) on the same pool, the
    first `pool_pairs` pairs of the mixed workload; its progress goes to this
    process's stderr."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serve",
           "--serve-pool", str(pool_pairs),
           "--serve-requests", str(args.serve_requests),
           "--serve-warmup", str(args.serve_warmup),
           "--serve-budget-gb", str(args.serve_budget_gb),
           "--serve-slots", str(args.serve_slots),
           "--serve-launch-pairs", str(args.serve_launch_pairs),
           "--serve-rates", args.serve_rates,
           "--serve-split", str(args.serve_split)]
    if args.serve_per_launch:
        cmd.append("--serve-per-launch")
    log("serve: in a process of its own: %s" % " ".join(cmd[2:]))
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=1800)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    # (exit 1 with a line: the served answers mismatched, which the block says)
    if r.returncode not in (0, 1) or not lines:
        raise RuntimeError("served-stream process failed (exit %d)" % r.returncode)
    blk = json.loads(lines[-1])["serve"]
    blk["process"] = "own process (bench.py --serve)"
    return blk


def serve_bench(args) -> int:
    """p50/p99 request latency of the served stream at fixed offered rates
    (its own JSON line; the default mixed-workload line carries the same
    block)."""
    from paper_2301_09310_amd import inputs as I
    from paper_2301_09310_amd import salo
    # latency bins: a served launch's requests wait for its longest pair,
    # which the throughput table's 16-lane groups run four times slower
    salo.load_tune_table(os.path.join(ROOT, "paper_2301_09310_amd", "tune_gfx950.json"),
                         "serve_bins")
    t0 = time.time()
    pool = I.mixed(0, args.serve_pool)
    log("serve pool: %d mixed pairs in %.1fs" % (pool.n_pairs, time.time() - t0))
    blk = serve_block(args, pool)
    blk["bin_table"] = "serve_bins of tune_gfx950.json (latency)"
    p99 = blk["rates"].get("0.8x", next(iter(blk["rates"].values())))["p99_ms"]
    rec = {"metric": METRIC, "value": p99, "unit": "ms (p99 at 0.8x)",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f16x2+u16x2",
           "config": {"workload": "served mixed requests", "pool_pairs": pool.n_pairs},
           "serve": blk}
    print(json.dumps(rec), flush=True)
    return 0 if blk["parity"] != "MISMATCH" else 1


if __name__ == "__main__":
    sys.exit(main())
