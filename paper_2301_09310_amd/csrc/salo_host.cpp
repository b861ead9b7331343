// Host side of the C ABI declared in include/salo.h: argument validation,
// per-(device, stream) workspaces and kernel launches.  Every step of the
// alignment itself runs in the gfx950 kernels (salo_kernels.hip).
#include <algorithm>
#include <mutex>
#include <map>
#include <vector>
#include <iterator>
#include <string>
#include <utility>
#include <cstdio>
#include <cstring>

#include "salo.h"
#include "salo_internal.h"

namespace salo {
namespace {

thread_local std::string g_last_error;

salo_status_t fail(salo_status_t st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

salo_status_t hip_fail(hipError_t e, const char *what) {
    return fail(SALO_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Workspace {
    int device = -1;
    int cus = 0;
    uint32_t *slab = nullptr;           // slot_words 32-bit words per slot
    int64_t slots = 0;
    int32_t slot_words = (int32_t)kSlotWords;
    unsigned long long *errors = nullptr;
    BinDesc *bins = nullptr;
    int32_t *counters = nullptr;        // kCounterWords: unit counters and totals per class
    // plan buffers of the persistent mode
    int64_t plan_cap = 0;               // pairs the plan buffers hold
    uint16_t *keys = nullptr;
    int32_t *order = nullptr;
    uint32_t *hist = nullptr;
    uint32_t *block_sums = nullptr;
    int32_t *binstat = nullptr;
    // optional timing events: [0] before plan, [1] before DP, [2] after DP
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool timed = false;
    bool timed_plan = false;
    // a call on this stream ran under stream capture: a graph may hold the
    // buffers' addresses, so growth keeps the old buffers (retired, freed
    // by salo_release) instead of freeing them
    bool captured = false;
    // carved from caller-provided device memory: never grows or frees
    bool external = false;
    std::vector<void *> retired;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// The (device, stream) workspace, created on first use.  Creation
// allocates the error counter, bin table and counters; it is recorded only
// once every allocation has succeeded (a failure frees what was made and
// leaves no entry).  It cannot happen under stream capture.
salo_status_t get_workspace(hipStream_t stream, Workspace **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, stream});
    if (it != g_ws.end()) {
        *out = &it->second;
        return SALO_OK;
    }
    if (capturing(stream))
        return fail(SALO_ERR_CAPTURE, "no workspace for this stream yet; call salo_reserve "
                                      "before capturing");
    Workspace w;
    w.device = dev;
    auto undo = [&](salo_status_t st, const std::string &msg) {
        if (w.errors) (void)hipFree(w.errors);
        if (w.bins) (void)hipFree(w.bins);
        if (w.counters) (void)hipFree(w.counters);
        return fail(st, msg);
    };
    e = hipDeviceGetAttribute(&w.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return undo(SALO_ERR_HIP, "hipDeviceGetAttribute");
    if (hipMalloc(&w.errors, sizeof(unsigned long long)) != hipSuccess) {
        w.errors = nullptr;
        return undo(SALO_ERR_NOMEM, "workspace: error counter");
    }
    if (hipMalloc(&w.bins, sizeof(BinDesc) * kMaxBins) != hipSuccess) {
        w.bins = nullptr;
        return undo(SALO_ERR_NOMEM, "workspace: bins");
    }
    if (hipMalloc(&w.counters, sizeof(int32_t) * kCounterWords) != hipSuccess) {
        w.counters = nullptr;
        return undo(SALO_ERR_NOMEM, "workspace: counters");
    }
    if ((e = hipMemset(w.errors, 0, sizeof(unsigned long long))) != hipSuccess)
        return undo(SALO_ERR_HIP, std::string("hipMemset: ") + hipGetErrorString(e));
    auto res = g_ws.emplace(std::make_pair(dev, stream), std::move(w));
    *out = &res.first->second;
    return SALO_OK;
}

// Free a buffer the workspace no longer uses, or keep it until
// salo_release when a captured graph may still use it.
void drop_buffer(Workspace &ws, void *p) {
    if (!p) return;
    if (ws.captured)
        ws.retired.push_back(p);
    else
        (void)hipFree(p);
}

salo_status_t grow_check(const Workspace &ws, hipStream_t stream, const char *what) {
    if (ws.external)
        return fail(SALO_ERR_INVALID, std::string(what) + " exceeds the fixed scratch");
    if (capturing(stream))
        return fail(SALO_ERR_CAPTURE, std::string(what) + " must grow during stream capture; "
                                                          "call salo_reserve first");
    return SALO_OK;
}

salo_status_t ensure_slots(Workspace &ws, int64_t slots, hipStream_t stream) {
    if (ws.slots >= slots) return SALO_OK;
    salo_status_t st = grow_check(ws, stream, "boundary slab");
    if (st != SALO_OK) return st;
    uint32_t *slab = nullptr;
    if (hipMalloc(&slab, (size_t)slots * (size_t)ws.slot_words * 4) != hipSuccess)
        return fail(SALO_ERR_NOMEM, "workspace: boundary slab of " +
                                        std::to_string(slots * ws.slot_words * 4) + " bytes");
    if (ws.slab) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            (void)hipFree(slab);
            return hip_fail(e, "hipStreamSynchronize");
        }
        drop_buffer(ws, ws.slab);
    }
    ws.slab = slab;
    ws.slots = slots;
    return SALO_OK;
}

salo_status_t ensure_plan(Workspace &ws, int64_t n_pairs, hipStream_t stream) {
    if (ws.plan_cap >= n_pairs && ws.hist) return SALO_OK;
    salo_status_t st = grow_check(ws, stream, "plan buffers");
    if (st != SALO_OK) return st;
    const int64_t cap = n_pairs < 1024 ? 1024 : n_pairs;
    uint16_t *keys = nullptr;
    int32_t *order = nullptr;
    uint32_t *hist = nullptr, *block_sums = nullptr;
    int32_t *binstat = nullptr;
    bool ok = hipMalloc(&keys, sizeof(uint16_t) * cap) == hipSuccess &&
              hipMalloc(&order, sizeof(int32_t) * cap) == hipSuccess;
    if (ok && !ws.hist)
        ok = hipMalloc(&hist, sizeof(uint32_t) * kHistEntries) == hipSuccess &&
             hipMalloc(&block_sums, sizeof(uint32_t) * kScanBlocks) == hipSuccess &&
             hipMalloc(&binstat, sizeof(int32_t) * 3 * kMaxBins) == hipSuccess;
    if (!ok) {
        for (void *q : {(void *)keys, (void *)order, (void *)hist, (void *)block_sums,
                        (void *)binstat})
            if (q) (void)hipFree(q);
        return fail(SALO_ERR_NOMEM, "workspace: plan buffers");
    }
    if (ws.keys || ws.order) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            for (void *q : {(void *)keys, (void *)order, (void *)hist, (void *)block_sums,
                            (void *)binstat})
                if (q) (void)hipFree(q);
            return hip_fail(e, "hipStreamSynchronize");
        }
        drop_buffer(ws, ws.keys);
        drop_buffer(ws, ws.order);
    }
    ws.keys = keys;
    ws.order = order;
    if (!ws.hist) {
        ws.hist = hist;
        ws.block_sums = block_sums;
        ws.binstat = binstat;
    }
    ws.plan_cap = cap;
    return SALO_OK;
}

// Length bins of the persistent mode: (m_hi, packed, lanes, cols).  Query-
// length ranges double from bin to bin; the built-in table is the
// autotuner's record for one MI355X (tune_gfx950.json), turned into
// kDefaultBins by the build, and can be replaced with salo_set_bins.
#include "salo_tune_table.inc"

std::mutex g_bins_mu;
std::vector<salo_bin_t> g_bins(std::begin(kDefaultBins), std::end(kDefaultBins));

// cols: forced query columns per lane for every bin, or 0 for each bin's
// own (its table entry; 0 there means 16).
BinTable make_bin_table(int cols, int forced_lanes) {
    std::lock_guard<std::mutex> lk(g_bins_mu);
    BinTable bt;
    std::memset(&bt, 0, sizeof bt);
    bt.n_bins = (int32_t)g_bins.size();
    int32_t prev_hi[2] = {0, 0};
    for (int b = 0; b < bt.n_bins; ++b) {
        const salo_bin_t &e = g_bins[b];
        bt.m_lo[b] = prev_hi[e.packed];
        bt.m_hi[b] = e.m_hi;
        prev_hi[e.packed] = e.m_hi;
        bt.packed[b] = e.packed;
        bt.lanes[b] = forced_lanes ? forced_lanes : e.lanes;
        bt.cols[b] = cols ? cols : (e.cols ? e.cols : 16);
    }
    return bt;
}

bool lanes_ok(int32_t w) {
    return w == 1 || w == 2 || w == 4 || w == 8 || w == 16 || w == 32 || w == 64;
}

salo_status_t validate(const uint8_t *q_seqs, const int64_t *q_offsets, const uint8_t *t_seqs,
                       const int64_t *t_offsets, int64_t n_pairs, salo_scoring_t sc,
                       const int32_t *os, const int32_t *oq, const int32_t *ot) {
    if (n_pairs < 0) return fail(SALO_ERR_INVALID, "n_pairs < 0");
    if (n_pairs > 0x7FFFFFFFll) return fail(SALO_ERR_INVALID, "n_pairs above 2^31-1");
    if (sc.match < 1 || sc.match > 32767)
        return fail(SALO_ERR_INVALID, "match must be in [1, 32767]");
    if (sc.mismatch > 0 || sc.mismatch < -32767)
        return fail(SALO_ERR_INVALID, "mismatch must be in [-32767, 0]");
    if (sc.gap_open < 0 || sc.gap_open > 32767)
        return fail(SALO_ERR_INVALID, "gap_open must be in [0, 32767]");
    if (sc.gap_extend < 0 || sc.gap_extend > 32767)
        return fail(SALO_ERR_INVALID, "gap_extend must be in [0, 32767]");
    if (n_pairs == 0) return SALO_OK;
    if (!q_seqs || !q_offsets || !t_seqs || !t_offsets || !os || !oq || !ot)
        return fail(SALO_ERR_INVALID, "NULL pointer argument");
    if (((uintptr_t)q_seqs & 3) || ((uintptr_t)t_seqs & 3))
        return fail(SALO_ERR_INVALID, "sequence streams must be 4-byte aligned");
    if (((uintptr_t)q_offsets & 7) || ((uintptr_t)t_offsets & 7))
        return fail(SALO_ERR_INVALID, "offset arrays must be 8-byte aligned");
    if (((uintptr_t)os & 3) || ((uintptr_t)oq & 3) || ((uintptr_t)ot & 3))
        return fail(SALO_ERR_INVALID, "output arrays must be 4-byte aligned");
    return SALO_OK;
}

// Shared by the forward and the start pass: option checks, workspace,
// KParams, then the plain or the persistent launch.  `starts` carries the
// forward answers for the start pass (nullptr for the forward pass).
struct StartArgs {
    const int32_t *score, *qend, *tend;
};
struct NMasks {
    const uint32_t *q, *t;   // either may be nullptr
};
// Per-request completion of the forward pass (salo_align_batch_tagged).
struct Signal {
    const int32_t *tag;
    uint32_t *done;
};
// Trace pass: the answers' starts, the CIGAR buffers and the code workspace.
struct TraceArgs {
    const int32_t *qstart, *tstart;
    const int64_t *cig_off;
    uint32_t *cig;
    int32_t *cig_len;
    uint8_t *ws;
    int64_t ws_bytes;
};

// Bins of the trace pass, for each cell kind, by span length.  Narrow
// lane groups put more pairs on a wave, and a wave walks its pairs' traces
// together, so they hide the walk's load latency best (measured on
// MI355X, short reads: 2 lanes 32.0 ms, 4 lanes 33.7, 16 lanes 47.1).
// But a wave's share of the workspace is split among its 64 / W groups, so
// a bin's width is raised until its longest span (rows taken as 1.5 x its
// length) fits a group's share: 0.5 B per cell and pair.
BinTable trace_bin_table(int cols, int forced_lanes, int64_t slot_bytes) {
    BinTable bt;
    std::memset(&bt, 0, sizeof bt);
    const int32_t hi[] = {16 * cols, 64 * cols, 256 * cols, 65535};
    const int32_t pref[] = {2, 8, 32, 64};
    int n = 0;
    for (int kind = 1; kind >= 0; --kind) {
        int32_t prev = 0;
        for (int b = 0; b < 4; ++b, ++n) {
            int w = pref[b];
            const double cells = 1.5 * (double)hi[b] * (double)hi[b];
            const double group_bytes = cells * (kind ? 1.0 : 0.5);   // two pairs or one
            while (w < 64 && (64.0 / w) * group_bytes > (double)slot_bytes) w <<= 1;
            bt.m_lo[n] = prev;
            bt.m_hi[n] = hi[b];
            prev = hi[b];
            bt.packed[n] = kind;
            bt.lanes[n] = forced_lanes ? forced_lanes : w;
            bt.cols[n] = cols;
        }
    }
    bt.n_bins = n;
    return bt;
}

// Lanes per pair group of the banded pass.  A chunk of W*K columns runs
// W*K + 2w rows (plus the W-1 step ramp) to cover its (2w+1)-wide stripe of
// the band, so narrow chunks compute fewer cells outside it; but a unit
// holds 128/W pairs, and a batch with too few units per resident wave ends
// on a long tail.  Measured on MI355X (200,000 anchored pairs of 500-5,000
// bases, bands 32..1000): chunks of max(32, w/4) columns rounded down to a
// power of two, and at least about two units per wave.
int band_lanes(int32_t band, int cols, int64_t n_pairs, int64_t grid) {
    const int64_t target = band / 4 > 32 ? band / 4 : 32;
    int w = 1;
    while (w < 64 && (int64_t)2 * w * cols <= target) w <<= 1;
    while (w < 64 && n_pairs * w < 2 * 128 * grid) w <<= 1;
    return w;
}

salo_status_t run_align(const uint8_t *q_seqs, const int64_t *q_offsets,
                        const uint8_t *t_seqs, const int64_t *t_offsets, int64_t n_pairs,
                        salo_scoring_t scoring, int32_t *out_score, int32_t *out_qend,
                        int32_t *out_tend, hipStream_t stream, const salo_options_t *opts,
                        const StartArgs *starts, NMasks masks, int32_t band = -1,
                        const TraceArgs *trace = nullptr, Workspace *ext = nullptr,
                        Signal sig = Signal{nullptr, nullptr}) {
    salo_options_t o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.split_waves != 0 && o.split_waves != 1 && o.split_waves != 4)
        return fail(SALO_ERR_INVALID, "split_waves must be 0, 1 or 4");
    const bool split = o.split_waves == 4;
    if (split && (starts || band >= 0 || trace || masks.q || masks.t))
        return fail(SALO_ERR_UNSUPPORTED, "split_waves applies to the forward pass only");
    if (o.no_f16 != 0 && o.no_f16 != 1) return fail(SALO_ERR_INVALID, "no_f16 must be 0 or 1");
    if (o.mode < SALO_MODE_AUTO || o.mode > SALO_MODE_PERSISTENT)
        return fail(SALO_ERR_INVALID, "unknown mode");
    if (o.waves_per_cu < 0 || o.waves_per_cu > 32)
        return fail(SALO_ERR_INVALID, "waves_per_cu must be in [0, 32]");
    if (starts && o.mode == SALO_MODE_PLAIN)
        return fail(SALO_ERR_UNSUPPORTED, "the start pass runs in persistent mode only");
    if (band >= 0 && o.mode == SALO_MODE_PLAIN)
        return fail(SALO_ERR_UNSUPPORTED, "the banded pass runs in persistent mode only");
    if (trace && o.mode == SALO_MODE_PLAIN)
        return fail(SALO_ERR_UNSUPPORTED, "the trace pass runs in persistent mode only");
    if (trace && o.cols != 0 && o.cols != 8 && o.cols != 16)
        return fail(SALO_ERR_UNSUPPORTED, "the trace pass supports cols 8 or 16");
    if (n_pairs == 0) return SALO_OK;

    Workspace *ws = ext;
    salo_status_t st = SALO_OK;
    if (!ws) {
        st = get_workspace(stream, &ws);
        if (st != SALO_OK) return st;
        if (capturing(stream)) ws->captured = true;
    }

    // resident waves per CU at the kernel's register budget: 3 per SIMD for
    // 8 or 16 query columns per lane, 2 per SIMD for 32
    const bool nm = masks.q != nullptr || masks.t != nullptr;
    // query columns per lane: 16, or 8 for a banded pass with a band of at
    // most 160 (measured: the narrower chunks it allows waste fewer cells)
    // (the trace pass: 16 columns, at 2 waves per SIMD, measured faster
    // than 8 at 3: 41.6 vs 51.6 ms for its fill on short reads)
    // (the default pass: each length bin's own column count, one persistent
    // launch per column class, 12 resident waves per CU for 8 or 16
    // columns, 8 for 32)
    const int cols_forced = o.cols ? o.cols
                                   : (band >= 0 ? (band <= 160 ? 8 : 16) : (trace ? 16 : 0));
    auto wpc_of = [&](int cols) {
        return o.waves_per_cu ? o.waves_per_cu : (cols >= 32 || (trace && cols > 8) ? 8 : 12);
    };
    const int one_cols = o.mode == SALO_MODE_PLAIN ? (o.cols ? o.cols : 16) : cols_forced;
    int64_t grid = (int64_t)ws->cus * (one_cols ? wpc_of(one_cols)
                                                : (o.waves_per_cu ? o.waves_per_cu : 12));
    if (ws->external && grid > ws->slots) grid = ws->slots;   // the fixed scratch's slots
    st = ensure_slots(*ws, grid, stream);
    if (st != SALO_OK) return st;

    KParams p;
    std::memset(&p, 0, sizeof p);
    p.q_seqs = q_seqs; p.q_off = q_offsets; p.t_seqs = t_seqs; p.t_off = t_offsets;
    p.n_pairs = n_pairs;
    p.match = scoring.match; p.mismatch = scoring.mismatch;
    p.gap_open = scoring.gap_open; p.gap_extend = scoring.gap_extend;
    p.out_score = out_score; p.out_qend = out_qend; p.out_tend = out_tend;
    if (starts) {
        p.in_score = starts->score; p.in_qend = starts->qend; p.in_tend = starts->tend;
    }
    p.order = nullptr;
    p.scratch = ws->slab;
    p.slot_words = ws->slot_words;
    // one pair group's column must fit a slot (banded units keep a ring of
    // rows, never more than the slot holds at this size)
    p.max_rows = band >= 0 ? (int32_t)SALO_MAX_LEN
                           : (int32_t)std::min<int64_t>(SALO_MAX_LEN, ws->slot_words / 2);
    p.errors = ws->errors;
    p.force_int32 = o.force_int32 ? 1 : 0;
    p.packed_ok = scoring_packed_ok(scoring.match, scoring.mismatch) ? 1 : 0;
    p.q_nmask = masks.q;
    p.t_nmask = masks.t;
    p.pair_tag = sig.tag;
    p.tag_done = sig.done;
    p.band = band;
    if (trace) {
        // each resident wave's share, at most 1 GiB (the kernel addresses
        // a share with 32-bit offsets)
        const int64_t slot =
            std::min<int64_t>(trace->ws_bytes / grid, (int64_t)1 << 30) & ~(int64_t)255;
        if (slot < 4096)
            return fail(SALO_ERR_INVALID, "trace workspace below 4 KiB per resident wave (" +
                                              std::to_string(grid) + " waves)");
        p.in_qstart = trace->qstart;
        p.in_tstart = trace->tstart;
        p.trace_ws = trace->ws;
        p.trace_slot = slot;
        p.cig_off = trace->cig_off;
        p.cig = trace->cig;
        p.cig_len = trace->cig_len;
        p.half_ok = 0;                 // choice bits need integer cells
    }
    // binary16 cells cannot give an N column the mismatch: off with masks
    p.half_ok = !o.no_f16 && !nm && scoring_half_ok(scoring.match, scoring.mismatch,
                                                    scoring.gap_open, scoring.gap_extend);
    p.bins = ws->bins;
    p.unit_counter = ws->counters;
    p.total_units = ws->counters + kColClasses;

    if (o.timing && ws->external)
        return fail(SALO_ERR_INVALID, "timing is not available on the fixed scratch");
    if (o.timing) {
        for (auto &ev : ws->ev)
            if (!ev && hipEventCreate(&ev) != hipSuccess)
                return fail(SALO_ERR_HIP, "hipEventCreate");
        ws->timed = true;
        ws->timed_plan = o.mode != SALO_MODE_PLAIN;
        if (hipEventRecord(ws->ev[0], stream) != hipSuccess)
            return fail(SALO_ERR_HIP, "hipEventRecord");
    }
    auto mark = [&](int k) -> salo_status_t {
        if (o.timing && hipEventRecord(ws->ev[k], stream) != hipSuccess)
            return fail(SALO_ERR_HIP, "hipEventRecord");
        return SALO_OK;
    };

    if (o.mode == SALO_MODE_PLAIN) {
        const int lanes = o.lanes ? o.lanes : 4;
        const int cols = o.cols ? o.cols : 16;
        if (!plain_variant_exists(lanes, cols))
            return fail(SALO_ERR_UNSUPPORTED, "no plain kernel for lanes=" +
                                                  std::to_string(lanes) + " cols=" +
                                                  std::to_string(cols));
        if ((st = mark(1)) != SALO_OK) return st;
        hipError_t e = launch_plain(p, lanes, cols, (int)grid, stream);
        if (e != hipSuccess) return hip_fail(e, "launch plain kernel");
        return mark(2);
    }

    // persistent, length-binned
    const int cols = cols_forced;
    if (cols != 0 && cols != 8 && cols != 16 && cols != 32)
        return fail(SALO_ERR_UNSUPPORTED, "persistent mode supports cols 8, 16 or 32");
    if (o.lanes && !persistent_lanes_supported(o.lanes))
        return fail(SALO_ERR_UNSUPPORTED, "persistent mode supports lanes 2..64");
    st = ensure_plan(*ws, n_pairs, stream);
    if (st != SALO_OK) return st;
    const BinTable bt =
        trace ? trace_bin_table(cols, o.lanes, p.trace_slot)
              : make_bin_table(cols, o.lanes ? o.lanes
                                             : (band >= 0 ? band_lanes(band, cols, n_pairs, grid)
                                                          : 0));
    // the split class takes the 16-bit bins of queries above 1024 bases,
    // in the split kernel's shape (64 lanes, 16 columns per lane)
    BinTable btx = bt;
    bool any_split = false;
    for (int b = 0; b < btx.n_bins; ++b) {
        btx.split[b] = split && btx.packed[b] && btx.m_lo[b] >= 1024 ? 1 : 0;
        if (btx.split[b]) {
            btx.lanes[b] = 64;
            btx.cols[b] = 16;
        }
        any_split = any_split || btx.split[b];
    }
    p.n_bins = btx.n_bins;
    PlanBuffers pb{ws->keys, ws->order, ws->hist, ws->block_sums, ws->binstat};
    hipError_t e = launch_plan(p, btx, pb, stream);
    if (e != hipSuccess) return hip_fail(e, "launch plan kernels");
    p.order = ws->order;
    if ((st = mark(1)) != SALO_OK) return st;
    // the split class first (its units are the longest), then one launch
    // per column class that a bin uses, widest first
    if (any_split) {
        // two resident 4-wave workgroups per CU (8 of the slots' waves)
        const int64_t g = std::min<int64_t>(grid, (int64_t)ws->cus * 8) / 4;
        e = launch_split(p, 16, 4, (int)g, stream);
        if (e != hipSuccess) return hip_fail(e, "launch split kernel");
    }
    bool used[kColClasses] = {false, false, false, false};
    for (int b = 0; b < btx.n_bins; ++b)
        if (!btx.split[b]) used[col_class(btx.cols[b])] = true;
    for (int k : {32, 16, 8}) {
        if (!used[col_class(k)]) continue;
        const int64_t g = std::min<int64_t>(grid, (int64_t)ws->cus * wpc_of(k));
        e = launch_persistent(p, k, (int)g, stream);
        if (e != hipSuccess) return hip_fail(e, "launch persistent kernel");
    }
    return mark(2);
}

}  // namespace

salo_status_t set_error(salo_status_t st, const char *msg) { return fail(st, msg); }

salo_status_t align_batch_fixed_scratch(const uint8_t *q_seqs, const int64_t *q_offsets,
                                        const uint8_t *t_seqs, const int64_t *t_offsets,
                                        int64_t n_pairs, salo_scoring_t scoring,
                                        int32_t *out_score, int32_t *out_qend,
                                        int32_t *out_tend, hipStream_t stream, void *scratch,
                                        int64_t scratch_bytes, int64_t max_pairs,
                                        int64_t slots, int32_t slot_words) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_score, out_qend, out_tend);
    if (st != SALO_OK) return st;
    if (n_pairs > max_pairs)
        return fail(SALO_ERR_INVALID, "n_pairs " + std::to_string(n_pairs) +
                                          " above the fixed scratch's maximum of " +
                                          std::to_string(max_pairs) + " pairs");
    if (n_pairs == 0) return SALO_OK;
    if (!scratch || (reinterpret_cast<uintptr_t>(scratch) & 255) ||
        scratch_bytes < fixed_scratch_bytes(max_pairs, slots, slot_words))
        return fail(SALO_ERR_INVALID, "fixed scratch missing, misaligned or too small");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Workspace w;
    w.device = dev;
    w.external = true;
    e = hipDeviceGetAttribute(&w.cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    char *c = static_cast<char *>(scratch);
    int64_t off = 0;
    auto carve = [&](int64_t bytes) {
        char *p = c + off;
        off += align256(bytes);
        return p;
    };
    w.counters = reinterpret_cast<int32_t *>(carve(4 * kCounterWords));
    // the plan's zeroing kernel clears every counter word at every call, so
    // the error counter (the two spare words) starts each call at 0
    w.errors = reinterpret_cast<unsigned long long *>(w.counters + 2 * kColClasses);
    w.bins = reinterpret_cast<BinDesc *>(carve((int64_t)sizeof(BinDesc) * kMaxBins));
    w.binstat = reinterpret_cast<int32_t *>(carve(12 * kMaxBins));
    w.block_sums = reinterpret_cast<uint32_t *>(carve(4 * (int64_t)kScanBlocks));
    w.hist = reinterpret_cast<uint32_t *>(carve(4 * kHistEntries));
    w.keys = reinterpret_cast<uint16_t *>(carve(2 * max_pairs));
    w.order = reinterpret_cast<int32_t *>(carve(4 * max_pairs));
    w.plan_cap = max_pairs;
    w.slab = reinterpret_cast<uint32_t *>(c + off);
    w.slots = slots;
    w.slot_words = slot_words;
    salo_options_t o;
    std::memset(&o, 0, sizeof o);
    o.mode = SALO_MODE_PERSISTENT;
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, out_score,
                     out_qend, out_tend, stream, &o, nullptr, NMasks{nullptr, nullptr}, -1,
                     nullptr, &w);
}

}  // namespace salo

using namespace salo;

extern "C" {

salo_status_t salo_align_batch_ex(const uint8_t *q_seqs, const int64_t *q_offsets,
                                  const uint8_t *t_seqs, const int64_t *t_offsets,
                                  int64_t n_pairs, salo_scoring_t scoring,
                                  int32_t *out_score, int32_t *out_qend, int32_t *out_tend,
                                  hipStream_t stream, const salo_options_t *opts) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_score, out_qend, out_tend);
    if (st != SALO_OK) return st;
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, out_score,
                     out_qend, out_tend, stream, opts, nullptr, NMasks{nullptr, nullptr});
}

salo_status_t salo_align_batch_n(const uint8_t *q_seqs, const uint32_t *q_nmask,
                                 const int64_t *q_offsets, const uint8_t *t_seqs,
                                 const uint32_t *t_nmask, const int64_t *t_offsets,
                                 int64_t n_pairs, salo_scoring_t scoring, int32_t *out_score,
                                 int32_t *out_qend, int32_t *out_tend, hipStream_t stream,
                                 const salo_options_t *opts) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_score, out_qend, out_tend);
    if (st != SALO_OK) return st;
    if ((reinterpret_cast<uintptr_t>(q_nmask) | reinterpret_cast<uintptr_t>(t_nmask)) & 3)
        return fail(SALO_ERR_INVALID, "N masks must be 4-byte aligned");
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, out_score,
                     out_qend, out_tend, stream, opts, nullptr, NMasks{q_nmask, t_nmask});
}

salo_status_t salo_align_starts(const uint8_t *q_seqs, const uint32_t *q_nmask,
                                const int64_t *q_offsets, const uint8_t *t_seqs,
                                const uint32_t *t_nmask, const int64_t *t_offsets,
                                int64_t n_pairs, salo_scoring_t scoring, const int32_t *score,
                                const int32_t *q_end, const int32_t *t_end,
                                int32_t *out_qstart, int32_t *out_tstart, hipStream_t stream,
                                const salo_options_t *opts) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_qstart, out_qstart, out_tstart);
    if (st != SALO_OK) return st;
    if (n_pairs > 0 && (!score || !q_end || !t_end))
        return fail(SALO_ERR_INVALID, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(score) | reinterpret_cast<uintptr_t>(q_end) |
         reinterpret_cast<uintptr_t>(t_end)) & 3)
        return fail(SALO_ERR_INVALID, "score / q_end / t_end must be 4-byte aligned");
    if ((reinterpret_cast<uintptr_t>(q_nmask) | reinterpret_cast<uintptr_t>(t_nmask)) & 3)
        return fail(SALO_ERR_INVALID, "N masks must be 4-byte aligned");
    const StartArgs sa{score, q_end, t_end};
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, nullptr,
                     out_qstart, out_tstart, stream, opts, &sa, NMasks{q_nmask, t_nmask});
}

salo_status_t salo_align_batch_banded(const uint8_t *q_seqs, const int64_t *q_offsets,
                                      const uint8_t *t_seqs, const int64_t *t_offsets,
                                      int64_t n_pairs, salo_scoring_t scoring, int32_t band,
                                      int32_t *out_score, int32_t *out_qend, int32_t *out_tend,
                                      hipStream_t stream, const salo_options_t *opts) {
    if (band < 0 || band > SALO_MAX_LEN)
        return fail(SALO_ERR_INVALID, "band must be in [0, 65535]");
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_score, out_qend, out_tend);
    if (st != SALO_OK) return st;
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, out_score,
                     out_qend, out_tend, stream, opts, nullptr, NMasks{nullptr, nullptr}, band);
}

salo_status_t salo_align_trace(const uint8_t *q_seqs, const int64_t *q_offsets,
                               const uint8_t *t_seqs, const int64_t *t_offsets, int64_t n_pairs,
                               salo_scoring_t scoring, const int32_t *score,
                               const int32_t *q_start, const int32_t *q_end,
                               const int32_t *t_start, const int32_t *t_end,
                               const int64_t *cigar_offsets, uint32_t *cigar,
                               int32_t *cigar_len, void *workspace, int64_t workspace_bytes,
                               hipStream_t stream, const salo_options_t *opts) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                cigar_len, cigar_len, cigar_len);
    if (st != SALO_OK) return st;
    if (n_pairs == 0) return SALO_OK;
    if (!score || !q_start || !q_end || !t_start || !t_end || !cigar_offsets || !cigar ||
        !workspace)
        return fail(SALO_ERR_INVALID, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(score) | reinterpret_cast<uintptr_t>(q_start) |
         reinterpret_cast<uintptr_t>(q_end) | reinterpret_cast<uintptr_t>(t_start) |
         reinterpret_cast<uintptr_t>(t_end) | reinterpret_cast<uintptr_t>(cigar)) & 3)
        return fail(SALO_ERR_INVALID, "answers and cigar must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(cigar_offsets) & 7)
        return fail(SALO_ERR_INVALID, "cigar_offsets must be 8-byte aligned");
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return fail(SALO_ERR_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes <= 0) return fail(SALO_ERR_INVALID, "workspace_bytes <= 0");
    const StartArgs sa{score, q_end, t_end};
    const TraceArgs ta{q_start, t_start, cigar_offsets, cigar, cigar_len,
                       static_cast<uint8_t *>(workspace), workspace_bytes};
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, nullptr, nullptr,
                     nullptr, stream, opts, &sa, NMasks{nullptr, nullptr}, -1, &ta);
}

salo_status_t salo_align_batch_tagged(const uint8_t *q_seqs, const int64_t *q_offsets,
                                      const uint8_t *t_seqs, const int64_t *t_offsets,
                                      int64_t n_pairs, salo_scoring_t scoring,
                                      int32_t *out_score, int32_t *out_qend, int32_t *out_tend,
                                      const int32_t *pair_tag, uint32_t *tag_done,
                                      hipStream_t stream, const salo_options_t *opts) {
    salo_status_t st = validate(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                                out_score, out_qend, out_tend);
    if (st != SALO_OK) return st;
    if (n_pairs > 0 && (!pair_tag || !tag_done))
        return fail(SALO_ERR_INVALID, "NULL pair_tag or tag_done");
    if ((reinterpret_cast<uintptr_t>(pair_tag) | reinterpret_cast<uintptr_t>(tag_done)) & 3)
        return fail(SALO_ERR_INVALID, "pair_tag and tag_done must be 4-byte aligned");
    return run_align(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring, out_score,
                     out_qend, out_tend, stream, opts, nullptr, NMasks{nullptr, nullptr}, -1,
                     nullptr, nullptr, Signal{pair_tag, tag_done});
}

salo_status_t salo_host_alloc(int64_t bytes, void **ptr) {
    if (!ptr || bytes <= 0) return fail(SALO_ERR_INVALID, "bytes <= 0 or NULL ptr");
    *ptr = nullptr;
    const hipError_t e = hipHostMalloc(ptr, (size_t)bytes, hipHostMallocCoherent);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(SALO_ERR_NOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    return SALO_OK;
}

salo_status_t salo_host_free(void *ptr) {
    if (!ptr) return SALO_OK;
    const hipError_t e = hipHostFree(ptr);
    if (e != hipSuccess) return hip_fail(e, "hipHostFree");
    return SALO_OK;
}

salo_status_t salo_align_batch(const uint8_t *q_seqs, const int64_t *q_offsets,
                               const uint8_t *t_seqs, const int64_t *t_offsets,
                               int64_t n_pairs, salo_scoring_t scoring, int32_t *out_score,
                               int32_t *out_qend, int32_t *out_tend, hipStream_t stream) {
    return salo_align_batch_ex(q_seqs, q_offsets, t_seqs, t_offsets, n_pairs, scoring,
                               out_score, out_qend, out_tend, stream, nullptr);
}

salo_status_t salo_reserve(int64_t max_pairs, hipStream_t stream) {
    if (max_pairs < 0) return fail(SALO_ERR_INVALID, "max_pairs < 0");
    Workspace *ws = nullptr;
    salo_status_t st = get_workspace(stream, &ws);
    if (st != SALO_OK) return st;
    st = ensure_slots(*ws, (int64_t)ws->cus * 12, stream);
    if (st != SALO_OK) return st;
    return ensure_plan(*ws, max_pairs, stream);
}

salo_status_t salo_error_count(hipStream_t stream, int64_t *host_count) {
    if (!host_count) return fail(SALO_ERR_INVALID, "host_count is NULL");
    Workspace *ws = nullptr;
    salo_status_t st = get_workspace(stream, &ws);
    if (st != SALO_OK) return st;
    unsigned long long v = 0;
    hipError_t e = hipMemcpyAsync(&v, ws->errors, sizeof v, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipMemsetAsync(ws->errors, 0, sizeof v, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *host_count = (int64_t)v;
    return SALO_OK;
}

salo_status_t salo_last_timing(hipStream_t stream, float *plan_ms, float *dp_ms) {
    if (!plan_ms || !dp_ms) return fail(SALO_ERR_INVALID, "NULL output pointer");
    Workspace *ws = nullptr;
    salo_status_t st = get_workspace(stream, &ws);
    if (st != SALO_OK) return st;
    if (!ws->timed) return fail(SALO_ERR_INVALID, "no timed call on this stream");
    hipError_t e = hipEventSynchronize(ws->ev[2]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float a = 0.f, b = 0.f;
    if ((e = hipEventElapsedTime(&a, ws->ev[0], ws->ev[1])) != hipSuccess ||
        (e = hipEventElapsedTime(&b, ws->ev[1], ws->ev[2])) != hipSuccess)
        return hip_fail(e, "hipEventElapsedTime");
    *plan_ms = ws->timed_plan ? a : 0.f;
    *dp_ms = b;
    return SALO_OK;
}

salo_status_t salo_set_bins(const salo_bin_t *bins, int32_t n_bins) {
    if (n_bins == 0 && bins == nullptr) {
        std::lock_guard<std::mutex> lk(g_bins_mu);
        g_bins.assign(std::begin(kDefaultBins), std::end(kDefaultBins));
        return SALO_OK;
    }
    if (!bins || n_bins < 2 || n_bins > kMaxBins)
        return fail(SALO_ERR_INVALID, "need 2..16 bins");
    int32_t prev[2] = {0, 0};
    bool last_full[2] = {false, false};
    int have[2] = {0, 0};
    for (int b = 0; b < n_bins; ++b) {
        const salo_bin_t &e = bins[b];
        if ((e.packed != 0 && e.packed != 1) || !lanes_ok(e.lanes) ||
            (e.cols != 0 && e.cols != 8 && e.cols != 16 && e.cols != 32))
            return fail(SALO_ERR_INVALID, "bin " + std::to_string(b) + ": bad packed/lanes/cols");
        if (e.m_hi <= prev[e.packed] || e.m_hi > SALO_MAX_LEN)
            return fail(SALO_ERR_INVALID, "bin " + std::to_string(b) +
                                              ": m_hi must increase within its kind");
        prev[e.packed] = e.m_hi;
        last_full[e.packed] = e.m_hi == SALO_MAX_LEN;
        have[e.packed]++;
    }
    if (!have[0] || !have[1] || !last_full[0] || !last_full[1])
        return fail(SALO_ERR_INVALID, "each kind needs bins ending at m_hi = 65535");
    std::lock_guard<std::mutex> lk(g_bins_mu);
    g_bins.assign(bins, bins + n_bins);
    return SALO_OK;
}

salo_status_t salo_get_bins(salo_bin_t *bins, int32_t max_bins, int32_t *n_bins) {
    if (!n_bins || (max_bins > 0 && !bins)) return fail(SALO_ERR_INVALID, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_bins_mu);
    *n_bins = (int32_t)g_bins.size();
    for (int b = 0; b < max_bins && b < (int)g_bins.size(); ++b) bins[b] = g_bins[b];
    return SALO_OK;
}

const char *salo_last_error(void) { return g_last_error.c_str(); }

void salo_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_ws) {
        Workspace &ws = kv.second;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(ws.device);
        (void)hipDeviceSynchronize();
        for (void *q : {(void *)ws.slab, (void *)ws.errors, (void *)ws.bins,
                        (void *)ws.counters, (void *)ws.keys, (void *)ws.order, (void *)ws.hist,
                        (void *)ws.block_sums, (void *)ws.binstat})
            if (q) (void)hipFree(q);
        for (void *q : ws.retired) (void)hipFree(q);
        for (auto ev : ws.ev)
            if (ev) (void)hipEventDestroy(ev);
        (void)hipSetDevice(cur);
    }
    g_ws.clear();
}

salo_status_t salo_pack_bases(const uint8_t *chars, int64_t n_chars, const int64_t *offsets,
                              int64_t n_seqs, int32_t revcomp, uint8_t *packed,
                              uint32_t *n_mask, unsigned long long *invalid_count,
                              hipStream_t stream) {
    if (n_chars < 0) return fail(SALO_ERR_INVALID, "n_chars < 0");
    if (n_seqs < 0) return fail(SALO_ERR_INVALID, "n_seqs < 0");
    if (revcomp != 0 && revcomp != 1) return fail(SALO_ERR_INVALID, "revcomp must be 0 or 1");
    if (n_chars == 0) return SALO_OK;
    if (!chars || !packed || (revcomp && !offsets))
        return fail(SALO_ERR_INVALID, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(chars) & 3) || (reinterpret_cast<uintptr_t>(packed) & 3))
        return fail(SALO_ERR_INVALID, "chars and packed must be 4-byte aligned");
    if (revcomp && (reinterpret_cast<uintptr_t>(offsets) & 7))
        return fail(SALO_ERR_INVALID, "offsets must be 8-byte aligned");
    if (invalid_count && (reinterpret_cast<uintptr_t>(invalid_count) & 7))
        return fail(SALO_ERR_INVALID, "invalid_count must be 8-byte aligned");
    if (n_mask && (reinterpret_cast<uintptr_t>(n_mask) & 3))
        return fail(SALO_ERR_INVALID, "n_mask must be 4-byte aligned");
    const hipError_t e = launch_pack(chars, n_chars, revcomp ? offsets : nullptr, n_seqs,
                                     revcomp != 0, packed, n_mask, invalid_count, stream);
    if (e != hipSuccess) return hip_fail(e, "launch pack kernel");
    return SALO_OK;
}

int32_t salo_version(void) { return SALO_VERSION; }

}  // extern "C"
