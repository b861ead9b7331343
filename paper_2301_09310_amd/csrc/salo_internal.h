// Internal interface between the host library (salo_host.cpp) and the
// gfx950 kernels (salo_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace salo {

// Boundary-column slab: one slot per resident wave.  A slot holds the
// chunk-boundary column (H and E of the last query column of a chunk, for
// every target row) of each pair group of the unit the wave is processing.
constexpr int64_t kSlotBytes = 512 * 1024;
constexpr int64_t kSlotWords = kSlotBytes / 4;

// Length bins of the persistent mode (by query length, and by target
// length so that every bin's boundary column fits a slot).
constexpr int kMaxBins = 8;
constexpr int64_t SALO_MAX_LEN_DEV = 65535;

struct BinDesc {
    int32_t lanes;        // lanes per pair group
    int32_t cols;         // query columns per lane
    int32_t packed;       // 1: 16-bit packed cells, 2 pairs per group
    int32_t pairs;        // pairs per unit
    int32_t count;        // pairs in this bin (device-written)
    int32_t first;        // first position of the bin in the sorted order
    int32_t units;        // units of this bin
    int32_t unit0;        // first global unit index of this bin
};

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
    uint32_t *scratch;             // kSlotWords words per slot, one slot per block
    unsigned long long *errors;    // invalid-pair counter
    int32_t force_int32;
    int32_t packed_ok;             // scoring admits 16-bit packed cells
    // persistent mode
    BinDesc *bins;                 // kMaxBins entries (device)
    int32_t n_bins;
    int32_t *unit_counter;         // atomic work counter
    int32_t *total_units;          // device-written
};

// Scoring admits the packed 16-bit path (match + |mismatch| fits a byte).
inline bool scoring_packed_ok(int32_t match, int32_t mismatch) {
    return match - mismatch <= 255;
}

hipError_t launch_plain(const KParams &p, int lanes, int cols, int grid,
                        hipStream_t stream);
bool plain_variant_exists(int lanes, int cols);

}  // namespace salo
