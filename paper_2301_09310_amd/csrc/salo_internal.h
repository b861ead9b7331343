// Internal interface between the host library (salo_host.cpp) and the
// gfx950 kernels (salo_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>
#include "salo.h"

namespace salo {

// Boundary-column slab: one slot per resident wave.  A slot holds the
// chunk-boundary column (H and E of the last query column of a chunk, for
// every target row) of each pair group of the unit the wave is processing.
constexpr int64_t kSlotBytes = 512 * 1024;
constexpr int64_t kSlotWords = kSlotBytes / 4;

// Length bins of the persistent mode (by query length, and by target
// length so that every bin's boundary column fits a slot).
constexpr int kMaxBins = 16;
constexpr int64_t SALO_MAX_LEN_DEV = 65535;

// One length bin: the pairs whose query length falls in (m_lo, m_hi] and
// whose score bound does (packed) or does not (wide) admit 16-bit cells.
struct BinDesc {
    int32_t lanes;        // lanes per pair group
    int32_t cols;         // query columns per lane
    int32_t packed;       // 1: 16-bit packed cells, 2 pairs per group
    int32_t pairs;        // pairs per unit (2 * 64 / lanes)
    int32_t count;        // pairs in this bin            (device-written)
    int32_t first;        // first sorted position        (device-written)
    int32_t units;        // units of this bin            (device-written)
    int32_t unit0;        // first global unit index      (device-written)
    int32_t n_min, n_max; // target length range          (device-written)
    int32_t split;        // 1: the split class runs this bin's units
};

// Query columns per lane (K) of a bin select one of three kernel
// instantiations; units are numbered within each such column class, and one
// persistent launch per class claims that class's units.  A fourth class,
// the split class, holds the bins whose units run on several waves each
// (salo_options_t.split_waves).
constexpr int kColClasses = 4;
constexpr int kSplitClass = 3;
__host__ __device__ inline int col_class(int cols) { return cols == 8 ? 0 : cols == 16 ? 1 : 2; }
__host__ __device__ inline int bin_class(int cols, int split) {
    return split ? kSplitClass : col_class(cols);
}
// unit counters [0, kColClasses), unit totals [kColClasses, 2 kColClasses),
// then two spare words (the fixed scratch's error counter)
constexpr int kCounterWords = 2 * kColClasses + 2;

// Static description of the bins, passed by value to the plan kernels.
struct BinTable {
    int32_t n_bins;
    int32_t m_lo[kMaxBins];    // lower query length of each bin (exclusive)
    int32_t m_hi[kMaxBins];    // upper query length of each bin (inclusive)
    int32_t packed[kMaxBins];  // 1: 16-bit bin, 0: 32-bit bin
    int32_t lanes[kMaxBins];
    int32_t cols[kMaxBins];
    int32_t split[kMaxBins];   // 1: units run by the split class (several waves each)
};

// Sort keys: bin (4 bits) | chunk count above the bin's minimum (4 bits,
// capped) | target length code (8 bits); pairs are processed in descending
// key order.
constexpr int kKeyBits = 16;
constexpr int kKeys = 1 << kKeyBits;
// The key histogram is split into kSubHist copies (a block uses copy
// blockIdx % kSubHist) so that concurrent increments rarely share an
// address; copies are laid out descending-key-major for one linear scan.
constexpr int kSubHist = 64;
constexpr int64_t kHistEntries = (int64_t)kKeys * kSubHist;
constexpr int kScanBlock = 4096;                        // entries per scan block
constexpr int kScanBlocks = (int)(kHistEntries / kScanBlock);

struct KParams {
    const uint8_t *q_seqs;
    const int64_t *q_off;
    const uint8_t *t_seqs;
    const int64_t *t_off;
    int64_t n_pairs;
    int32_t match, mismatch, gap_open, gap_extend;
    int32_t *out_score;
    int32_t *out_qend;
    int32_t *out_tend;
    const int32_t *order;          // processing order of pair ids (nullptr: identity)
    uint32_t *scratch;             // slot_words words per slot, one slot per block
    int32_t slot_words;            // boundary-slot size (kSlotWords unless the caller's
                                   // scratch is smaller)
    int32_t max_rows;              // longest column (target rows) a slot holds for one
                                   // pair group; longer pairs are flagged invalid
    unsigned long long *errors;    // invalid-pair counter
    // start-position pass: the forward answers (score, q_end, t_end) of each
    // pair; the pass aligns the reversed prefixes ending there and writes
    // q_start / t_start to out_qend / out_tend (nullptr: the forward pass)
    const int32_t *in_score;
    const int32_t *in_qend;
    const int32_t *in_tend;
    // optional N masks (bit k of word k>>5 marks base k of the stream as N;
    // an N scores mismatch against every base); nullptr: no N
    const uint32_t *q_nmask;
    const uint32_t *t_nmask;
    // banded pass: only cells with |i - j| <= band exist (-1: no band)
    int32_t band;
    // trace pass (with in_score / in_qend / in_tend): the answers' starts;
    // the pass aligns q[q_start..q_end] against t[t_start..t_end], keeps a
    // 4-bit choice code per cell in trace_ws (trace_slot bytes per block)
    // and writes each pair's CIGAR runs to cig[cig_off[p] ..], their count
    // to cig_len[p] (nullptr cig: not the trace pass)
    const int32_t *in_qstart;
    const int32_t *in_tstart;
    uint8_t *trace_ws;
    int64_t trace_slot;
    const int64_t *cig_off;
    uint32_t *cig;
    int32_t *cig_len;
    // per-request completion (forward pass): after pair p's outputs are
    // written, tag_done[pair_tag[p]] is incremented with a system-scope
    // release (nullptr pair_tag: no signal; a negative tag: none for p)
    const int32_t *pair_tag;
    uint32_t *tag_done;
    int32_t force_int32;
    int32_t packed_ok;             // scoring admits 16-bit packed cells
    int32_t half_ok;               // scoring admits binary16 cells (and no_f16 is off)
    // persistent mode
    BinDesc *bins;                 // kMaxBins entries (device)
    int32_t n_bins;
    // per column class (kColClasses: 8, 16, 32 query columns per lane):
    // the atomic work counter and the unit count of that class's bins
    int32_t *unit_counter;         // [kColClasses]
    int32_t *total_units;          // [kColClasses], device-written
};

// Scoring admits the packed 16-bit path (match + |mismatch| fits a byte).
inline bool scoring_packed_ok(int32_t match, int32_t mismatch) {
    return match - mismatch <= 255;
}

// Largest value a packed 16-bit cell may take: below 0x7C00 every cell
// value, read as a binary16 number, is finite and non-negative, so the
// packed half-precision maximum orders cells exactly like integers.
constexpr int32_t kPackedLimit = 0x7BFF;

// A pair fits 16-bit cells when its best score plus one substitution step
// stays within kPackedLimit (every H, E, F and diagonal sum is below that).
__host__ __device__ inline bool packed_bound_ok(int32_t match, int32_t mismatch, int64_t mn) {
    return (int64_t)match * (mn + 1) - (int64_t)mismatch <= kPackedLimit;
}

// binary16 holds every integer of magnitude <= 2048 exactly.  A pair runs
// in binary16 cells when its best score is at most that: every
// non-negative value the recurrence forms is then exact, and a negative
// one, rounded or not, stays negative and loses every maximum against the
// zero-clamped E.
constexpr int32_t kHalfExact = 2048;
__host__ __device__ inline bool half_bound_ok(int32_t match, int64_t mn) {
    return (int64_t)match * mn <= kHalfExact;
}

// The binary16 row table stores one byte per score: the high byte of its
// binary16 encoding, so the low byte must be 0.  That holds for integers
// with at most three significant bits (1..8, 10, 12, 14, 16, 20, ...);
// alpha and beta must be exact too.
inline bool half_value_ok(int32_t v) {
    const uint32_t a = (uint32_t)(v < 0 ? -v : v);
    if (a > (uint32_t)kHalfExact) return false;
    uint32_t top = a;
    int drop = 0;
    while (top >= 8u) {
        top >>= 1;
        ++drop;
    }
    return (top << drop) == a;
}
inline bool scoring_half_ok(int32_t match, int32_t mismatch, int32_t gap_open,
                            int32_t gap_extend) {
    return half_value_ok(match) && half_value_ok(mismatch) &&
           (int64_t)gap_open + gap_extend <= kHalfExact && gap_extend <= kHalfExact;
}

// Boundary-slot rows of a banded unit with R target rows.  A chunk reads
// its left neighbour's column only on rows c0-w-1 .. c0-1+w (2w+1 rows), so
// a ring of 2w+2 rows, rounded up to a power of two, holds them; *wrap is
// the ring's row mask.  A unit with no more rows than that keeps every row
// (mask all ones).
__host__ __device__ inline int band_slot_rows(int R, int w, uint32_t *wrap) {
    int64_t ring = 1;
    while (ring < 2 * (int64_t)w + 2) ring <<= 1;
    if (ring >= R) {
        *wrap = 0xFFFFFFFFu;
        return R;
    }
    *wrap = (uint32_t)ring - 1u;
    return (int)ring;
}

// A fixed scratch buffer carved into the persistent path's workspace (the
// no-allocation entry point): counters (kCounterWords words, the error
// counter in the two spare ones), bin table, bin statistics, scan block sums, key histogram,
// keys and order for max_pairs pairs, then `slots` boundary slots of
// slot_words words.  Every part starts on a 256-byte boundary.
constexpr int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }
constexpr int64_t fixed_scratch_bytes(int64_t max_pairs, int64_t slots, int64_t slot_words) {
    return align256(4 * kCounterWords) + align256((int64_t)sizeof(BinDesc) * kMaxBins) +
           align256(12 * kMaxBins) + align256(4 * (int64_t)kScanBlocks) +
           align256(4 * kHistEntries) + align256(2 * max_pairs) + align256(4 * max_pairs) +
           slots * slot_words * 4;
}

// Record `msg` as the calling thread's salo_last_error() text; returns st.
salo_status_t set_error(salo_status_t st, const char *msg);

// Align a batch (salo_align_batch's arguments and behaviour) with every
// workspace buffer carved from `scratch` (device memory of scratch_bytes
// bytes laid out as fixed_scratch_bytes describes).  Allocates nothing.
// More than max_pairs pairs: SALO_ERR_INVALID.
salo_status_t align_batch_fixed_scratch(const uint8_t *q_seqs, const int64_t *q_offsets,
                                        const uint8_t *t_seqs, const int64_t *t_offsets,
                                        int64_t n_pairs, salo_scoring_t scoring,
                                        int32_t *out_score, int32_t *out_qend,
                                        int32_t *out_tend, hipStream_t stream, void *scratch,
                                        int64_t scratch_bytes, int64_t max_pairs,
                                        int64_t slots, int32_t slot_words);

hipError_t launch_plain(const KParams &p, int lanes, int cols, int grid,
                        hipStream_t stream);
hipError_t launch_persistent(const KParams &p, int cols, int grid, hipStream_t stream);
// the split class: workgroups of `waves` waves (4), 16 columns per lane
hipError_t launch_split(const KParams &p, int cols, int waves, int grid, hipStream_t stream);
hipError_t launch_pack(const uint8_t *chars, int64_t n_chars, const int64_t *offsets,
                       int64_t n_seqs, bool revcomp, uint8_t *packed, uint32_t *n_mask,
                       unsigned long long *invalid, hipStream_t stream);
bool persistent_lanes_supported(int lanes);

struct PlanBuffers {
    uint16_t *keys;        // [n_pairs]
    int32_t *order;        // [n_pairs] pair ids in processing order
    uint32_t *hist;        // [kHistEntries] counts, then cursors
    uint32_t *block_sums;  // [kScanBlocks]
    int32_t *binstat;      // [kMaxBins * 3]: count, n_min, n_max
};

// Plan: bins, keys, counting sort by key (descending) and the unit table.
hipError_t launch_plan(const KParams &p, const BinTable &bt, const PlanBuffers &pb,
                       hipStream_t stream);
bool plain_variant_exists(int lanes, int cols);

}  // namespace salo
