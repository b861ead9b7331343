/*
 * salo.h -- C ABI of the MI355X (gfx950) batched seed-extension library.
 *
 * The operation (SALoBa, arXiv 2301.09310, Section II-A, Eq. 1): for every
 * (query, target) pair of a batch, fill the affine-gap Smith-Waterman-Gotoh
 * table
 *     H(i,j) = max{0, E(i,j), F(i,j), H(i-1,j-1) + S(i,j)}
 *     E(i,j) = max{H(i,j-1) - alpha, E(i,j-1) - beta}
 *     F(i,j) = max{H(i-1,j) - alpha, F(i-1,j) - beta}
 * with i over target (reference) bases and j over query bases, and return
 * the maximum H over the table and its position (Section II-A, Eq. 1).  Batches of pairs of uneven length are the workload of
 * Section III-A (load imbalance) and Section V-D.
 *
 * Scoring (salo_scoring_t): S(i,j) = match when the bases are equal and
 * mismatch otherwise; a gap of k bases costs gap_open + k*gap_extend, i.e.
 * alpha = gap_open + gap_extend, beta = gap_extend.  Constraints:
 * 1 <= match <= 32767, -32767 <= mismatch <= 0, 0 <= gap_open <= 32767,
 * 0 <= gap_extend <= 32767.
 *
 * Sequence layout: bases A=0, C=1, G=2, T=3, 2 bits each, base k of a
 * stream in byte k>>2 at bits 2*(k&3) (least significant pair first).
 * q_seqs and t_seqs are two independent streams; pair p uses query bases
 * [q_offsets[p], q_offsets[p+1]) and target bases
 * [t_offsets[p], t_offsets[p+1]).  Offsets are int64, in bases, and need
 * not be byte aligned.  Each stream pointer must be 4-byte aligned, its
 * buffer readable up to the next multiple of 4 bytes past its last base,
 * and hold at most 2^32-4 bytes.  Lengths are limited to 65535 bases.
 *
 * Results: out_score[p] >= 0; out_qend[p] / out_tend[p] are the 0-based
 * query / target indices of the highest cell, the first one in row-major
 * order (smallest target index, then smallest query index) when several
 * cells tie; both are -1 when the score is 0.  A pair with invalid device
 * data (decreasing offsets, or a length above 65535) gets -1 in all three
 * outputs and is counted (salo_error_count).
 *
 * Memory and ownership: every pointer argument of the align calls is a
 * DEVICE pointer on the current HIP device.  The caller owns inputs and
 * outputs and keeps them alive until `stream` has passed the call; inputs
 * are never written and the three outputs are fully overwritten.  The
 * library owns a workspace per (device, stream), grown on demand outside
 * stream capture (salo_reserve pre-sizes it; a call under capture that
 * needs a larger workspace, or the first call on a stream made under
 * capture, returns SALO_ERR_CAPTURE and enqueues nothing).  Once a call on
 * a stream has been captured into a graph, the buffers that graph uses are
 * never freed before salo_release(), even when a later, larger call on the
 * stream grows the workspace, so the graph stays valid to replay.
 *
 * Errors and synchronisation: host-checkable errors return a negative
 * status and enqueue nothing (NULL pointer with n_pairs > 0, n_pairs < 0,
 * scoring out of range, misaligned stream pointer, n_pairs above 2^31-1);
 * a failed HIP call returns SALO_ERR_HIP.  salo_last_error() gives a
 * thread-local message for the last non-OK status.  n_pairs == 0 is a
 * no-op.  The align calls are asynchronous: they only enqueue work on
 * `stream` and never synchronise it.  Calls on different streams may run
 * concurrently; calls that share a stream share its workspace in order.
 */
#ifndef SALO_H
#define SALO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SALO_VERSION 1
#define SALO_MAX_LEN 65535

typedef struct {
    int32_t match;       /* score of equal bases, > 0 */
    int32_t mismatch;    /* score of unequal bases, <= 0 */
    int32_t gap_open;    /* gap of k bases costs gap_open + k*gap_extend */
    int32_t gap_extend;
} salo_scoring_t;

typedef enum {
    SALO_OK = 0,
    SALO_ERR_INVALID = -1,   /* bad argument (host-checkable) */
    SALO_ERR_NOMEM = -2,     /* workspace allocation failed */
    SALO_ERR_HIP = -3,       /* a HIP runtime call failed */
    SALO_ERR_CAPTURE = -4,   /* workspace must grow while the stream is captured */
    SALO_ERR_UNSUPPORTED = -5
} salo_status_t;

typedef enum {
    SALO_MODE_AUTO = 0,        /* persistent, length-binned (the default) */
    SALO_MODE_PLAIN = 1,       /* one launch, pairs in input order, fixed lanes/cols */
    SALO_MODE_PERSISTENT = 2   /* one persistent launch over length bins */
} salo_mode_t;

typedef struct {
    int32_t mode;           /* salo_mode_t */
    int32_t lanes;          /* lanes per pair group (1,2,4,8,16,32,64); 0 = default */
    int32_t cols;           /* query columns per lane (8, 16 or 32); 0 = default
                               (each length bin's own, persistent mode) */
    int32_t force_int32;    /* 1: 32-bit cells for every pair */
    int32_t waves_per_cu;   /* grid size in resident waves per CU; 0 = default */
    int32_t timing;         /* 1: record events around the plan and DP kernels
                               (see salo_last_timing); 0 = off */
    int32_t no_f16;         /* 1: never use binary16 cells (16-bit integer or
                               32-bit cells only); results are identical */
    int32_t split_waves;    /* 0 or 1: off.  4: the pairs of the 16-bit bins of
                               queries above 1024 bases run with 64 lanes and
                               16 columns per lane, each unit on 4 waves of
                               one workgroup, one strip of target rows each,
                               so a long pair finishes sooner (forward pass,
                               persistent mode; for latency, e.g. serving a
                               batch with fewer long pairs than the GPU has
                               SIMDs).  Results are identical.  Other values:
                               SALO_ERR_INVALID. */
} salo_options_t;

/* One length bin of the persistent mode: pairs whose query length is at
 * most m_hi (and above the previous bin's m_hi of the same kind), with
 * 16-bit cells (packed = 1; binary16 or 16-bit integer cells, chosen per
 * unit of work from its pairs' score bounds) or 32-bit cells (packed = 0), run in lane
 * groups of `lanes` lanes.  A pair whose target is too long for its bin's
 * width (more than 1024 * lanes bases) moves to the next bin of its kind. */
typedef struct {
    int32_t m_hi;       /* 1..65535, increasing within each kind */
    int32_t packed;     /* 1: 16-bit bin, 0: 32-bit bin */
    int32_t lanes;      /* 1, 2, 4, 8, 16, 32 or 64 */
    int32_t cols;       /* query columns per lane: 8, 16 or 32; 0 means 16 */
} salo_bin_t;

#define SALO_MAX_BINS 16

/*
 * Align n_pairs pairs (Eq. 1 of Section II-A per pair) with default options.
 * Arguments: packed query stream, its int64 offsets [n_pairs+1], packed
 * target stream, its offsets [n_pairs+1], pair count, scoring, three int32
 * output arrays [n_pairs], and the HIP stream to enqueue on.
 */
salo_status_t salo_align_batch(const uint8_t *q_seqs, const int64_t *q_offsets,
                               const uint8_t *t_seqs, const int64_t *t_offsets,
                               int64_t n_pairs, salo_scoring_t scoring,
                               int32_t *out_score, int32_t *out_qend,
                               int32_t *out_tend, hipStream_t stream);

/*
 * As salo_align_batch, with explicit execution options (opts may be NULL).
 * Every mode and every lanes/cols choice returns identical results; they
 * differ only in how work is mapped to the GPU (Section IV-A's intra-query
 * parallelism and Section IV-C's subwarp width are the lanes choice).
 */
salo_status_t salo_align_batch_ex(const uint8_t *q_seqs, const int64_t *q_offsets,
                                  const uint8_t *t_seqs, const int64_t *t_offsets,
                                  int64_t n_pairs, salo_scoring_t scoring,
                                  int32_t *out_score, int32_t *out_qend,
                                  int32_t *out_tend, hipStream_t stream,
                                  const salo_options_t *opts);

/*
 * As salo_align_batch_ex, for reads with unknown bases (N; the paper's
 * five-letter reads, Section II-B).  q_nmask / t_nmask: DEVICE uint32
 * arrays, 4-byte aligned, one bit per base of the stream (bit k of word k>>5
 * set: base k is N; its 2-bit code is ignored), covering
 * ceil(offsets[n_pairs] / 32) words; either may be NULL (no N in that
 * stream).  An N scores `mismatch` against every base, N included.  With a
 * mask the 16-bit integer and 32-bit cells are used (binary16 cells are
 * off).
 */
salo_status_t salo_align_batch_n(const uint8_t *q_seqs, const uint32_t *q_nmask,
                                 const int64_t *q_offsets, const uint8_t *t_seqs,
                                 const uint32_t *t_nmask, const int64_t *t_offsets,
                                 int64_t n_pairs, salo_scoring_t scoring, int32_t *out_score,
                                 int32_t *out_qend, int32_t *out_tend, hipStream_t stream,
                                 const salo_options_t *opts);

/*
 * Start positions of the answers of a previous align call: where the
 * optimal path to the highest cell (Section II-A) begins.  For every pair
 * with score > 0 ending at (q_end, t_end), out_qstart / out_tstart receive
 * the first aligned pair of an optimal alignment ending there; among
 * several optimal starts, the one with the largest t_start, then the
 * largest q_start.  Computed as the first maximum of Eq. 1 over the
 * reversed prefixes q[q_end..0], t[t_end..0] (it equals the score exactly
 * at the optimal starts, because (q_end, t_end) is the first maximum of the
 * whole table).
 * Arguments: the align call's sequences, N masks (NULL for none, see
 * salo_align_batch_n), offsets, n_pairs and scoring; its
 * three outputs score, q_end, t_end (DEVICE int32 [n_pairs], 4-byte
 * aligned); out_qstart, out_tstart (DEVICE int32 [n_pairs], fully
 * overwritten; -1 for pairs with score 0).  A pair whose given answer is
 * not Eq. 1's (its reversed prefixes' best score differs, or the end lies
 * outside the pair) gets -1 in both and is counted (salo_error_count).
 * Runs the persistent mode (opts->mode = SALO_MODE_PLAIN returns
 * SALO_ERR_UNSUPPORTED); other options and all errors as
 * salo_align_batch_ex.
 */
salo_status_t salo_align_starts(const uint8_t *q_seqs, const uint32_t *q_nmask,
                                const int64_t *q_offsets, const uint8_t *t_seqs,
                                const uint32_t *t_nmask, const int64_t *t_offsets,
                                int64_t n_pairs, salo_scoring_t scoring, const int32_t *score,
                                const int32_t *q_end, const int32_t *t_end,
                                int32_t *out_qstart, int32_t *out_tstart, hipStream_t stream,
                                const salo_options_t *opts);

/*
 * Banded alignment (Section VII-B: seed extension often fills only the
 * cells within a fixed distance of the main diagonal).  Eq. 1 over the
 * cells with |i - j| <= band only, i indexing target bases and j query
 * bases; a cell outside the band acts as the table's boundary (H = 0, no
 * gap open from it) and is never the answer.  Outputs as
 * salo_align_batch: the highest in-band score and the first (row-major)
 * in-band cell holding it; (0, -1, -1) when no in-band cell scores above
 * 0.  A band of at least max(query, target length) - 1 gives
 * salo_align_batch's answer.
 * band: 0..65535 (else SALO_ERR_INVALID).  Other arguments, options and
 * errors as salo_align_batch_ex; runs the persistent mode
 * (opts->mode = SALO_MODE_PLAIN returns SALO_ERR_UNSUPPORTED).  With
 * opts->cols = 0 the query columns per lane are 8 for a band of at most
 * 160, else 16.  With opts->lanes = 0 the lane-group width W is chosen from the band and the
 * batch: the largest power of two with W * cols <= max(64, band / 2), raised
 * (up to 64) until the batch fills about two units of work per resident
 * wave (a unit holds 128 / W pairs).
 */
salo_status_t salo_align_batch_banded(const uint8_t *q_seqs, const int64_t *q_offsets,
                                      const uint8_t *t_seqs, const int64_t *t_offsets,
                                      int64_t n_pairs, salo_scoring_t scoring, int32_t band,
                                      int32_t *out_score, int32_t *out_qend,
                                      int32_t *out_tend, hipStream_t stream,
                                      const salo_options_t *opts);

/*
 * Trace of the best alignment (Section II-A: the path that reaches the
 * highest cell), as a run-length CIGAR, for the answers of an align call
 * and a start call on the same inputs and scoring.  For every pair with
 * score > 0, one optimal alignment from (q_start, t_start) to
 * (q_end, t_end); when several are optimal, the one chosen walking back from
 * the end by preferring, at every step, an aligned pair over an I over a D,
 * and inside a gap, the gap opening at this base over it extending.
 * Runs are written in alignment order to cigar[cigar_offsets[p] ..] as
 * uint32 (length << 4) | op with BAM codes: 7 '=' (equal bases), 8 'X'
 * (unequal bases), 1 'I' (query base against a gap in the target), 2 'D'
 * (target base against a gap in the query).
 * Arguments: the align call's sequences, offsets, n_pairs and scoring; the
 * answers score, q_start, q_end, t_start, t_end (DEVICE int32 [n_pairs],
 * 4-byte aligned); cigar_offsets (DEVICE int64 [n_pairs + 1], 8-byte
 * aligned; pair p owns cigar[cigar_offsets[p] .. cigar_offsets[p+1]), and
 * q_end - q_start + t_end - t_start + 1 runs always suffice); cigar (DEVICE
 * uint32); cigar_len (DEVICE int32 [n_pairs], fully overwritten: the run
 * count, 0 for score 0, -1 for a pair whose answers are not Eq. 1's or
 * whose runs do not fit, -2 for a pair too large for its share of the
 * workspace; -1 and -2 are counted, see salo_error_count).
 * workspace: DEVICE scratch of workspace_bytes, 256-byte aligned, owned by
 * the caller and only used during the call.  Each resident wave (CUs x 8
 * with the default 16 columns per lane, CUs x 12 with opts->cols = 8)
 * gets an equal share, at most 1 GiB (bytes past that are not used); a wave
 * aligns up to 64 / W pair groups at once (a group holds two pairs in
 * 16-bit cells or one in 32-bit cells) and each group needs ceil(its
 * longer span / (W x cols)) x W x cols x (its longer span's rows) / 2 bytes
 * of it per pair.  W (2..64 lanes) grows with the span length, and with
 * opts->lanes = 0 also until a span length class fits the workspace, so a
 * larger workspace gives narrower, faster groups.  Too small for 4 KiB per
 * wave: SALO_ERR_INVALID.
 * Runs in the persistent mode with 16-bit integer cells where the score
 * bound allows and 32-bit cells elsewhere (opts->force_int32 forces the
 * latter; opts->mode = SALO_MODE_PLAIN or opts->cols = 32 return
 * SALO_ERR_UNSUPPORTED); other options and errors as salo_align_batch_ex.
 */
salo_status_t salo_align_trace(const uint8_t *q_seqs, const int64_t *q_offsets,
                               const uint8_t *t_seqs, const int64_t *t_offsets, int64_t n_pairs,
                               salo_scoring_t scoring, const int32_t *score,
                               const int32_t *q_start, const int32_t *q_end,
                               const int32_t *t_start, const int32_t *t_end,
                               const int64_t *cigar_offsets, uint32_t *cigar,
                               int32_t *cigar_len, void *workspace, int64_t workspace_bytes,
                               hipStream_t stream, const salo_options_t *opts);

/* Pre-size the workspace of (current device, stream) for batches of up to
 * max_pairs pairs, so later calls allocate nothing (needed before graph
 * capture).  Synchronous with respect to the host. */
salo_status_t salo_reserve(int64_t max_pairs, hipStream_t stream);

/* Number of invalid pairs seen on (current device, stream) since the last
 * call; synchronises `stream`, then resets the counter. */
salo_status_t salo_error_count(hipStream_t stream, int64_t *host_count);

/* Durations of the last align call on (current device, stream) that ran
 * with opts->timing = 1: the planning kernels (binning and sorting; 0 in
 * plain mode) and the DP kernel, in milliseconds, from HIP events recorded
 * on `stream` around those launches.  Synchronises on the events.  Returns
 * SALO_ERR_INVALID when no timed call has run on that stream. */
salo_status_t salo_last_timing(hipStream_t stream, float *plan_ms, float *dp_ms);

/* Replace the process-wide length-bin table of the persistent mode (the
 * lane-group width per query-length bin, normally written by the
 * autotuner).  bins may be NULL with n_bins == 0 to restore the built-in
 * table.  Each kind (16-bit, 32-bit) needs at least one bin and its last
 * bin must have m_hi = 65535.  Applies to calls made after it returns;
 * results never depend on the table. */
salo_status_t salo_set_bins(const salo_bin_t *bins, int32_t n_bins);

/* Copy the current bin table into bins[0 .. max_bins-1]; *n_bins receives
 * the table's length. */
salo_status_t salo_get_bins(salo_bin_t *bins, int32_t max_bins, int32_t *n_bins);

/*
 * Pack character reads into the 2-bit stream the align calls read (reads
 * carry one byte per base, SALoBa Section II-B; the evaluation packs them
 * on the device for every method, Section V-A).
 *
 * chars: DEVICE, n_chars bytes, the concatenated sequences, 4-byte aligned
 *   and readable up to the next multiple of 4 bytes.  A, C, G, T are
 *   accepted in either case; N and n too when n_mask is given; any other
 *   byte is an invalid base, written as A (0) and counted.
 * offsets: DEVICE int64 [n_seqs+1], 8-byte aligned, the sequences' CSR in
 *   characters (non-decreasing, offsets[0] = 0, offsets[n_seqs] = n_chars).
 *   Read only when revcomp = 1 (it may be NULL otherwise).
 * revcomp: 0 = output base k is chars[k]; 1 = each sequence is reverse-
 *   complemented in place: output base k of sequence s is the complement
 *   (A<->T, C<->G) of chars[offsets[s] + offsets[s+1] - 1 - k].  With
 *   revcomp a base no sequence covers (offsets breaking the rule above) is
 *   written as A and counted.
 * packed: DEVICE, 4-byte aligned, ceil(n_chars/16)*4 bytes, fully
 *   overwritten (base k in byte k>>2 at bits 2*(k&3); bits past the last
 *   base are 0).  It must not overlap chars.  The output offsets of the
 *   sequences equal the input offsets (one base per character), so
 *   (packed, offsets) can be passed straight to the align calls.
 * n_mask: DEVICE uint32 [ceil(n_chars/32)], 4-byte aligned, or NULL: bit k
 *   of word k>>5 is set when output base k is N (its 2-bit code is 0); the
 *   complement of N is N.  (packed, n_mask) go straight to
 *   salo_align_batch_n.
 * invalid_count: DEVICE counter or NULL; the kernel adds the number of
 *   invalid bases to it (the caller clears it).
 * Asynchronous on `stream`; host-checkable errors (n_chars < 0, NULL or
 * misaligned pointers, revcomp not 0/1, n_seqs < 0) return
 * SALO_ERR_INVALID and enqueue nothing; n_chars == 0 is a no-op.
 */
salo_status_t salo_pack_bases(const uint8_t *chars, int64_t n_chars, const int64_t *offsets,
                              int64_t n_seqs, int32_t revcomp, uint8_t *packed,
                              uint32_t *n_mask, unsigned long long *invalid_count,
                              hipStream_t stream);

/*
 * salo_align_batch_ex with per-request completion, for serving several
 * requests merged into one call: pair p belongs to request pair_tag[p]
 * (DEVICE int32 [n_pairs]; a negative tag means no request), and once
 * pair p's three outputs are written the library adds 1 to
 * tag_done[pair_tag[p]], so a host thread that reads tag_done[r] == (pairs
 * of request r) can read that request's outputs while the rest of the call
 * still runs.  tag_done and the three output arrays must be host memory
 * from salo_host_alloc: the device writes the outputs through to it and
 * issues each count after those stores have completed.  tag_done must hold
 * every tag used, and the caller zeroes the counters before the call.
 * Counters that share a 128-byte line contend (the device's increments of
 * one line are serialised): give each request a line of its own, e.g. tags
 * 32 apart.  Outputs in device memory are written as usual, but the counts
 * then do not order them for the host: read them after the stream has
 * passed the call.  Arguments, options, layout and errors otherwise as
 * salo_align_batch_ex (NULL pair_tag or tag_done with n_pairs > 0:
 * SALO_ERR_INVALID).
 */
salo_status_t salo_align_batch_tagged(const uint8_t *q_seqs, const int64_t *q_offsets,
                                      const uint8_t *t_seqs, const int64_t *t_offsets,
                                      int64_t n_pairs, salo_scoring_t scoring,
                                      int32_t *out_score, int32_t *out_qend, int32_t *out_tend,
                                      const int32_t *pair_tag, uint32_t *tag_done,
                                      hipStream_t stream, const salo_options_t *opts);

/* Pinned host memory that the host and the device both read and write
 * coherently (hipHostMalloc with the coherent flag), for salo_align_batch_
 * tagged's counters and outputs; *ptr is usable on the host and, as the
 * same address, in device calls.  salo_host_free releases it (no call may
 * still use it).  bytes <= 0 or NULL ptr: SALO_ERR_INVALID; failure:
 * SALO_ERR_NOMEM. */
salo_status_t salo_host_alloc(int64_t bytes, void **ptr);
salo_status_t salo_host_free(void *ptr);

/*
 * salo_align_batch without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, serving loops
 * that must not call hipMalloc, harnesses that forbid it.  Same arguments,
 * layout, results and asynchrony as salo_align_batch, and the same kernels;
 * the workspace is one fixed device array inside the library (about
 * 328 MiB, held by each GPU the library runs on until the process ends),
 * found with hipGetSymbolAddress on the first call on each device.
 *
 * Limits: n_pairs <= 4,194,304 (else SALO_ERR_INVALID, nothing enqueued);
 * a pair whose target exceeds 12,288 bases gets -1 in all three outputs
 * (as do pairs with invalid offsets or lengths); no error counter is kept.
 * Every call on one GPU shares that array and leaves its contents behind:
 * calls that overlap on a GPU (on different streams, or from different
 * host threads) race and must be serialised by the caller.  Calls on one
 * stream are ordered and safe.
 */
salo_status_t salo_align_batch_noalloc(const uint8_t *q_seqs, const int64_t *q_offsets,
                                       const uint8_t *t_seqs, const int64_t *t_offsets,
                                       int64_t n_pairs, salo_scoring_t scoring,
                                       int32_t *out_score, int32_t *out_qend,
                                       int32_t *out_tend, hipStream_t stream);

/* Message for the last non-OK status returned on this host thread. */
const char *salo_last_error(void);

/* Free every workspace the library holds (no call may be in flight). */
void salo_release(void);

/* SALO_VERSION of the loaded library. */
int32_t salo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SALO_H */
