// Host side of the C ABI declared in include/salo.h: argument validation,
// per-(device, stream) workspaces and kernel launches.  Every step of the
// alignment itself runs in the gfx950 kernels (salo_kernels.hip).
#include <mutex>
#include <map>
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
    uint32_t *slab = nullptr;           // kSlotBytes per slot
    int64_t slots = 0;
    unsigned long long *errors = nullptr;
    BinDesc *bins = nullptr;
    int32_t *counters = nullptr;        // [0] unit counter, [1] total units
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

salo_status_t get_workspace(hipStream_t stream, Workspace **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &ws = g_ws[{dev, stream}];
    if (ws.device < 0) {
        ws.device = dev;
        e = hipDeviceGetAttribute(&ws.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        e = hipMalloc(&ws.errors, sizeof(unsigned long long));
        if (e != hipSuccess) return fail(SALO_ERR_NOMEM, "workspace: error counter");
        e = hipMemset(ws.errors, 0, sizeof(unsigned long long));
        if (e != hipSuccess) return hip_fail(e, "hipMemset");
        e = hipMalloc(&ws.bins, sizeof(BinDesc) * kMaxBins);
        if (e != hipSuccess) return fail(SALO_ERR_NOMEM, "workspace: bins");
        e = hipMalloc(&ws.counters, sizeof(int32_t) * 4);
        if (e != hipSuccess) return fail(SALO_ERR_NOMEM, "workspace: counters");
    }
    *out = &ws;
    return SALO_OK;
}

bool capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

salo_status_t ensure_slots(Workspace &ws, int64_t slots, hipStream_t stream) {
    if (ws.slots >= slots) return SALO_OK;
    if (capturing(stream))
        return fail(SALO_ERR_CAPTURE, "workspace must grow during stream capture; "
                                      "call salo_reserve first");
    if (ws.slab) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        hipFree(ws.slab);
        ws.slab = nullptr;
        ws.slots = 0;
    }
    hipError_t e = hipMalloc(&ws.slab, (size_t)slots * kSlotBytes);
    if (e != hipSuccess) {
        ws.slab = nullptr;
        return fail(SALO_ERR_NOMEM, "workspace: boundary slab of " +
                                        std::to_string(slots * kSlotBytes) + " bytes");
    }
    ws.slots = slots;
    return SALO_OK;
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

}  // namespace
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
    salo_options_t o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    for (int r : o.reserved)
        if (r != 0) return fail(SALO_ERR_INVALID, "salo_options_t.reserved must be 0");
    if (o.mode < SALO_MODE_AUTO || o.mode > SALO_MODE_PERSISTENT)
        return fail(SALO_ERR_INVALID, "unknown mode");
    if (o.waves_per_cu < 0 || o.waves_per_cu > 32)
        return fail(SALO_ERR_INVALID, "waves_per_cu must be in [0, 32]");
    if (n_pairs == 0) return SALO_OK;

    Workspace *ws = nullptr;
    st = get_workspace(stream, &ws);
    if (st != SALO_OK) return st;

    const int wpc = o.waves_per_cu ? o.waves_per_cu : 8;
    const int64_t grid = (int64_t)ws->cus * wpc;
    st = ensure_slots(*ws, grid, stream);
    if (st != SALO_OK) return st;

    KParams p;
    std::memset(&p, 0, sizeof p);
    p.q_seqs = q_seqs; p.q_off = q_offsets; p.t_seqs = t_seqs; p.t_off = t_offsets;
    p.n_pairs = n_pairs;
    p.match = scoring.match; p.mismatch = scoring.mismatch;
    p.gap_open = scoring.gap_open; p.gap_extend = scoring.gap_extend;
    p.out_score = out_score; p.out_qend = out_qend; p.out_tend = out_tend;
    p.order = nullptr;
    p.scratch = ws->slab;
    p.errors = ws->errors;
    p.force_int32 = o.force_int32 ? 1 : 0;
    p.packed_ok = scoring_packed_ok(scoring.match, scoring.mismatch) ? 1 : 0;
    p.bins = ws->bins;
    p.unit_counter = ws->counters;
    p.total_units = ws->counters + 1;

    // Until the binned persistent path lands, every mode runs the plain kernel.
    const int lanes = o.lanes ? o.lanes : 4;
    const int cols = o.cols ? o.cols : 16;
    if (!plain_variant_exists(lanes, cols))
        return fail(SALO_ERR_UNSUPPORTED, "no kernel variant for lanes=" +
                                              std::to_string(lanes) + " cols=" +
                                              std::to_string(cols));
    hipError_t e = launch_plain(p, lanes, cols, (int)grid, stream);
    if (e != hipSuccess) return hip_fail(e, "launch plain kernel");
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
    return ensure_slots(*ws, (int64_t)ws->cus * 8, stream);
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

const char *salo_last_error(void) { return g_last_error.c_str(); }

void salo_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_ws) {
        Workspace &ws = kv.second;
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(ws.device);
        hipDeviceSynchronize();
        if (ws.slab) hipFree(ws.slab);
        if (ws.errors) hipFree(ws.errors);
        if (ws.bins) hipFree(ws.bins);
        if (ws.counters) hipFree(ws.counters);
        hipSetDevice(cur);
    }
    g_ws.clear();
}

int32_t salo_version(void) { return SALO_VERSION; }

}  // extern "C"
