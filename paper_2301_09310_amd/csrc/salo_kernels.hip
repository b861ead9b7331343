// gfx950 kernels for batched affine-gap seed extension.
//
// Operation (SALoBa, arXiv 2301.09310, Section II-A, Eq. 1): per pair, the
// Smith-Waterman-Gotoh table over target rows i and query columns j, and
// the first (row-major) cell holding its maximum.
//
// Mapping to CDNA4 (differs from the paper's CUDA design, Section IV):
//  * A "group" of W lanes of a wave64 works on one pair (or two, see
//    below) as a linear systolic array: lane l holds K query columns of the
//    current chunk in VGPRs; target rows stream through the group; at step
//    s lane l computes row s-l.  H and E of a lane's last column move to
//    lane l+1 with one DPP row/wave shift (the paper passes them through
//    shared memory, Section IV-A; it also found shuffles no faster,
//    Section VII-A -- here the DPP move replaces both).  A chunk is W*K
//    query columns; the group sweeps chunks left to right, and the last
//    lane's column of a chunk (H and E for every row) is written to a
//    per-wave global slot that lane 0 reads back, 4 rows ahead, for the
//    next chunk (the role of the paper's lazy spill, Section IV-B).
//  * Cells are 16-bit where a pair's score bound allows it: two pairs share
//    a group, one in each half of every VGPR, and every DP operation is one
//    packed instruction (v_pk_add_u16 / v_pk_sub_u16 clamp / v_pk_max_u16,
//    and v_pk_maximum3_f16 as an exact three-way integer maximum: see
//    pmax3).
//    E and F are clamped at 0; any E/F value <= 0 yields the same H, so
//    unsigned saturating subtraction is exact.  The substitution score comes
//    from one v_perm_b32 per cell pair: a per-row byte table (match -
//    mismatch at the target base's slot) indexed by per-column query
//    selectors.  Pairs outside the 16-bit bound use 32-bit cells, one pair
//    per group.
//  * Narrow groups (small W) are the paper's subwarps (Section IV-C):
//    several pairs share a wave; the lanes-per-group choice trades the
//    wavefront's ramp against column padding and per-wave imbalance.
//  * End positions follow the first-maximum rule exactly: a lane keeps the
//    highest row maximum of its columns with the first row reaching it
//    (strict comparison), saves that row's H values to LDS when it
//    improves, and at the end of a chunk finds the first column holding the
//    maximum.  Candidates merge lexicographically (score, -row, -col)
//    across chunks and then across the group's lanes.
//
// All lane-group counts and loop bounds of a unit are wave-uniform; units
// never wait on one another, so every wave runs to completion on its own.
#include "salo_internal.h"

namespace salo {
namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_v(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t psub(uint32_t a, uint32_t b) {
    return as_u(__builtin_elementwise_sub_sat(as_v(a), as_v(b)));
}
__device__ __forceinline__ uint32_t padd(uint32_t a, uint32_t b) {
    return as_u(as_v(a) + as_v(b));
}
__device__ __forceinline__ uint32_t pmax(uint32_t a, uint32_t b) {
    return as_u(__builtin_elementwise_max(as_v(a), as_v(b)));
}
// a * b + c in both halves (v_pk_mad_u16)
__device__ __forceinline__ uint32_t pmad(uint32_t a, uint32_t b, uint32_t c) {
    return as_u(as_v(a) * as_v(b) + as_v(c));
}
// 1 in each half that is non-zero, else 0, given one = 0x00010001
__device__ __forceinline__ uint32_t pnz(uint32_t a, uint32_t one) {
    return as_u(__builtin_elementwise_min(as_v(a), as_v(one)));
}
// A constant the optimiser cannot see through (the empty asm emits no
// instruction).  With literal operands it rewrites min(x, 1) into a compare
// and a * 16 + c into a shift and an or, and with no packed 16-bit compare
// it then splits both into per-half compares, selects and repacking; with
// these operands pnz and pmad stay one packed instruction each.
__device__ __forceinline__ uint32_t opaque(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}
// A value the reassociation pass cannot look into (no instruction): the
// code word's Horner step acc * 16 + nibble then stays one multiply-add,
// where distributing the nibble's own sum over it would take four.
__device__ __forceinline__ uint32_t sealed(uint32_t v) {
    asm("" : "+v"(v));
    return v;
}
// Maximum of three packed cell pairs.  Cell values stay in [0, 0x7BFF]
// (kPackedLimit), where reading the bits as binary16 gives finite,
// non-negative numbers (denormals included, which the kernels keep) in the
// same order as the integers; the half-precision maximum returns one of
// its operands unchanged, so one v_pk_maximum3_f16 is an exact integer
// max3 for both halves.
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pmax3(uint32_t a, uint32_t b, uint32_t c) {
    const f16x2 x = __builtin_bit_cast(f16x2, a);
    const f16x2 y = __builtin_bit_cast(f16x2, b);
    const f16x2 z = __builtin_bit_cast(f16x2, c);
    return __builtin_bit_cast(
        uint32_t, __builtin_elementwise_maximum(__builtin_elementwise_maximum(x, y), z));
}
// binary16 cells: exact integer arithmetic on values of magnitude <= 2048
__device__ __forceinline__ uint32_t hadd(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t,
                              __builtin_bit_cast(f16x2, a) + __builtin_bit_cast(f16x2, b));
}
__device__ __forceinline__ uint32_t hmax(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(
                                            __builtin_bit_cast(f16x2, a),
                                            __builtin_bit_cast(f16x2, b)));
}
__device__ __forceinline__ int32_t half_bits_to_int(uint32_t v) {
    return (int32_t)(float)__builtin_bit_cast(_Float16, (uint16_t)v);
}
__device__ __forceinline__ int max3i(int a, int b, int c) {
    return max(max(a, b), c);
}

constexpr int kWave = 64;
constexpr int32_t kBufDword3 = 0x00020000;   // raw buffer descriptor, gfx9 family

// A packed base stream behind a range-checked buffer descriptor: reads
// outside [0, nbytes) return 0 instead of touching memory.
struct BaseStream {
    const uint8_t *base;   // wave-uniform
    int32_t nbytes;        // wave-uniform, whole 32-bit words

    __device__ __forceinline__ void init(const uint8_t *p, const int64_t *off, int64_t n_pairs) {
        int64_t bases = n_pairs > 0 ? off[n_pairs] : 0;
        int64_t bytes = ((bases + 15) >> 4) << 2;
        if (bytes < 0) bytes = 0;
        if (bytes > 0xFFFFFFF0ll) bytes = 0xFFFFFFF0ll;
        base = p;
        nbytes = __builtin_amdgcn_readfirstlane((int)(uint32_t)bytes);
    }
    // an N-mask stream: one bit per base, 32 bases per word
    __device__ __forceinline__ void init_mask(const uint32_t *p, const int64_t *off,
                                              int64_t n_pairs) {
        int64_t bases = (p != nullptr && n_pairs > 0) ? off[n_pairs] : 0;
        int64_t bytes = ((bases + 31) >> 5) << 2;
        if (bytes < 0) bytes = 0;
        if (bytes > 0xFFFFFFF0ll) bytes = 0xFFFFFFF0ll;
        base = reinterpret_cast<const uint8_t *>(p);
        nbytes = __builtin_amdgcn_readfirstlane((int)(uint32_t)bytes);
    }
    // the 32 mask bits of bases pos .. pos+31 (bit 0 = base pos)
    __device__ __forceinline__ uint32_t bits32(int64_t pos) const {
        const int64_t w = pos >> 5;
        return __builtin_amdgcn_alignbit(word(w + 1), word(w), (uint32_t)(pos & 31));
    }
    __device__ __forceinline__ uint32_t word(int64_t w) const {
        // the descriptor is rebuilt from scalar values at every use so that
        // it stays in SGPRs (no waterfall loop)
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(base), 0, nbytes, kBufDword3);
        const uint32_t off = (w < 0 || w >= (int64_t(1) << 30)) ? 0xFFFFFFF0u
                                                                : (uint32_t)w << 2;
        return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off, 0, 0);
    }
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The wave's boundary-column slot behind a range-checked buffer descriptor
// of `bytes`: a byte offset at or past the end reads 0 and drops the store
// (the hardware checks the offset against the descriptor's size).  Entries
// are 8 bytes, (H, E), at byte offset 8 * (row * groups + group).
struct Slot {
    uint32_t *base;   // wave-uniform
    uint32_t bytes;   // wave-uniform

    __device__ __forceinline__ uint2 load(uint32_t off) const {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kBufDword3);
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        return make_uint2(v.x, v.y);
    }
    __device__ __forceinline__ void store(uint32_t off, uint32_t h, uint32_t e) const {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kBufDword3);
        u32x2 v;
        v.x = h;
        v.y = e;
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
    }
    // 16 bytes per lane: one burst of the LDS ring (64 lanes x 16 B = 1 KiB)
    __device__ __forceinline__ uint4 load16(uint32_t off) const {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kBufDword3);
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    __device__ __forceinline__ void store16(uint32_t off, uint4 v) const {
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kBufDword3);
        u32x4 w;
        w.x = v.x;
        w.y = v.y;
        w.z = v.z;
        w.w = v.w;
        __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)off, 0, 0);
    }
};

// The chunk-boundary column in LDS (the role of the paper's lazy spill,
// Section IV-B, designed for one wave64 and its LDS).  A pair group's
// column holds (H, E) of the chunk's last query column for every target
// row, 8 bytes per row, laid out [row][group] as in the global slot.
//  * Resident: a unit whose whole column fits kBndLdsBytes keeps it in LDS;
//    the next chunk reads each row before this chunk overwrites it (the
//    read of row r leads its write by W steps), so one buffer serves both.
//  * Ring: otherwise the column lives in the wave's global slot and LDS
//    holds two rings of two 1 KiB blocks (a block is 128 / Gs rows of all
//    Gs groups).  The writer side stores each row into the write ring and,
//    when a block is complete, the whole wave copies it to the slot as one
//    coalesced 16-byte-per-lane burst.  The reader side keeps the next block
//    in flight in four registers per lane and moves it into the read ring
//    one block ahead of use.  So the slot sees 2 bursts per block instead of
//    a load and a store per row, and each row is read from LDS.
constexpr uint32_t kBndLdsBytes = 4096;
constexpr uint32_t kBndBlockBytes = 1024;
// a wave clears the region with four 16-byte stores per lane
static_assert(kBndLdsBytes == 4 * kBndBlockBytes && kBndBlockBytes == 16 * kWave,
              "boundary column layout");

__device__ __forceinline__ uint2 lds_load8(const uint32_t *lds, uint32_t byte_off) {
    return *reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(lds) + byte_off);
}
__device__ __forceinline__ void lds_store8(uint32_t *lds, uint32_t byte_off, uint32_t h,
                                           uint32_t e) {
    *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(lds) + byte_off) = make_uint2(h, e);
}
__device__ __forceinline__ uint4 lds_load16(const uint32_t *lds, uint32_t byte_off) {
    return *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(lds) + byte_off);
}
__device__ __forceinline__ void lds_store16(uint32_t *lds, uint32_t byte_off, uint4 v) {
    *reinterpret_cast<uint4 *>(reinterpret_cast<char *>(lds) + byte_off) = v;
}
// Order this wave's LDS (and global) accesses across lanes: everything
// before is complete before anything after starts.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// DPP move of `v` from lane-1 to every lane (wave_shr:1), with `bnd` at
// each group's first lane (l == 0), whatever the group width.
__device__ __forceinline__ uint32_t shift_in(uint32_t v, uint32_t bnd, bool first) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138, 0xf, 0xf, true);
    return first ? bnd : s;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, kWave));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t group_max_u64(uint64_t v, int W) {
    for (int o = W >> 1; o >= 1; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, kWave);
        const uint64_t w = ((uint64_t)hi << 32) | lo;
        v = w > v ? w : v;
    }
    return v;
}

struct PairRef {
    int64_t q0, t0;
    int32_t m, n;
    int32_t id;       // original pair index, -1 when absent
    bool invalid;
};

// The pair at position `pos` of the processing order, or an absent pair
// (no output, m = n = 0) when pos is outside [0, pos_end).
// REV (start pass): the pair's reversed prefixes ending at its forward
// answer (q_end, t_end): m = q_end + 1, n = t_end + 1, and q0 / t0 are the
// stream positions of the reversed sequences' first bases (q_end, t_end);
// a pair with forward score 0 is empty.
// TR (trace pass): the span q[q_start..q_end] x t[t_start..t_end] of the
// pair's answer; a pair with score 0 is empty.
template <bool REV, bool TR = false>
__device__ __forceinline__ PairRef load_pair(const KParams &P, int64_t pos, int64_t pos_end,
                                             bool present) {
    PairRef r{0, 0, 0, 0, -1, false};
    if (!present || pos < 0 || pos >= pos_end || pos >= P.n_pairs) return r;
    const int64_t p = P.order ? (int64_t)P.order[pos] : pos;
    if (p < 0 || p >= P.n_pairs) return r;     // never for a consistent plan
    const int64_t q0 = P.q_off[p], q1 = P.q_off[p + 1];
    const int64_t t0 = P.t_off[p], t1 = P.t_off[p + 1];
    r.id = (int32_t)p;
    const int64_t m = q1 - q0, n = t1 - t0;
    if (m < 0 || n < 0 || m > SALO_MAX_LEN_DEV || n > SALO_MAX_LEN_DEV || q0 < 0 || t0 < 0) {
        r.invalid = true;
        return r;
    }
    if constexpr (REV) {
        const int32_t sc = P.in_score[p], qe = P.in_qend[p], te = P.in_tend[p];
        if (sc <= 0) return r;
        if (qe < 0 || qe >= m || te < 0 || te >= n) {
            r.invalid = true;
            return r;
        }
        r.q0 = q0 + qe; r.t0 = t0 + te; r.m = qe + 1; r.n = te + 1;
    } else if constexpr (TR) {
        const int32_t sc = P.in_score[p], qe = P.in_qend[p], te = P.in_tend[p];
        const int32_t qs = P.in_qstart[p], ts = P.in_tstart[p];
        if (sc <= 0) return r;
        if (qs < 0 || qs > qe || qe >= m || ts < 0 || ts > te || te >= n) {
            r.invalid = true;
            return r;
        }
        r.q0 = q0 + qs; r.t0 = t0 + ts; r.m = qe - qs + 1; r.n = te - ts + 1;
    } else {
        r.q0 = q0; r.t0 = t0; r.m = (int32_t)m; r.n = (int32_t)n;
    }
    // a column longer than one group's share of the slot cannot be held
    if (r.n > P.max_rows) {
        r.q0 = r.t0 = 0;
        r.m = r.n = 0;
        r.invalid = true;
    }
    return r;
}

// Reverse the order of the sixteen 2-bit bases of a word.
__device__ __forceinline__ uint32_t rev2(uint32_t x) {
    const uint32_t r = __builtin_bitreverse32(x);      // bases reversed, bit pairs swapped
    return ((r >> 1) & 0x55555555u) | ((r & 0x55555555u) << 1);
}

struct Best {
    int32_t score, row, col;
    __device__ __forceinline__ void offer(int32_t s, int32_t r, int32_t c) {
        if (s > score || (s == score && s > 0 && (r < row || (r == row && c < col)))) {
            score = s; row = r; col = c;
        }
    }
    __device__ __forceinline__ uint64_t key() const {
        if (score <= 0) return 0;
        return ((uint64_t)(uint32_t)score << 32) | ((uint64_t)(0xFFFFu - (uint32_t)row) << 16) |
               (uint64_t)(0xFFFFu - (uint32_t)col);
    }
};

// Forward pass: score and end.  Start pass (REV): the reversed prefixes'
// best cell (j', i') must score the forward answer; q_start = q_end - j',
// t_start = t_end - i' go to out_qend / out_tend (a pair whose reversed
// maximum differs from the given score, or whose end lies outside it, is
// counted as invalid and gets -1).
template <bool REV>
__device__ __forceinline__ void write_result(const KParams &P, const PairRef &pr, uint64_t key) {
    if (pr.id < 0) return;
    if constexpr (REV) {
        const int32_t s = (int32_t)(key >> 32);
        const int32_t want = P.in_score[pr.id];
        if (pr.invalid || (want > 0 && s != want)) {
            P.out_qend[pr.id] = -1; P.out_tend[pr.id] = -1;
            atomicAdd(P.errors, 1ull);
            return;
        }
        const int32_t jr = (int32_t)(0xFFFFu - (uint32_t)(key & 0xFFFF));
        const int32_t ir = (int32_t)(0xFFFFu - (uint32_t)((key >> 16) & 0xFFFF));
        P.out_qend[pr.id] = s > 0 ? (pr.m - 1) - jr : -1;
        P.out_tend[pr.id] = s > 0 ? (pr.n - 1) - ir : -1;
        return;
    }
    // System-scope stores write through the L2, so that signal_done can
    // announce them to the host without writing back the whole L2 (12 bytes
    // per pair; device-memory outputs take the same path).
    const int32_t s = pr.invalid ? -1 : (int32_t)(key >> 32);
    const int32_t qe = pr.invalid ? -1 : s > 0 ? (int32_t)(0xFFFFu - (uint32_t)(key & 0xFFFF)) : -1;
    const int32_t te =
        pr.invalid ? -1 : s > 0 ? (int32_t)(0xFFFFu - (uint32_t)((key >> 16) & 0xFFFF)) : -1;
    __hip_atomic_store(P.out_score + pr.id, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(P.out_qend + pr.id, qe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(P.out_tend + pr.id, te, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (pr.invalid) atomicAdd(P.errors, 1ull);
}

// Per-request completion: count pair `id` as finished for its tag.  The
// outputs and the counters live in coherent host memory (salo_host_alloc).
// write_result stored the outputs at system scope (through the L2); once
// those stores have completed they are visible to the host, and the count
// that announces them is issued only then.  (A release fence at system
// scope would do the same by writing back the whole L2 at every call.)
__device__ __forceinline__ void signal_done(const KParams &P, int32_t id) {
    if (P.pair_tag == nullptr || id < 0) return;
    const int32_t tg = P.pair_tag[id];
    if (tg >= 0) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __hip_atomic_fetch_add(P.tag_done + tg, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Trace pass: choice codes, one nibble per cell, as the fill stores them.
// Bit 0: H is not the diagonal term; bit 1: H is not E (so the walk takes
// the diagonal, then E, then F, whichever first gives H); bit 2: E extends
// E(i, j-1) rather than opening from H(i, j-1) (open is taken on equal
// values); bit 3: F extends F(i-1, j) likewise.  Every bit is "a != b"
// for values with a >= b, which 16-bit unsigned cells compute as
// min(a - b, 1) in both halves at once.
// Layouts, per group and chunk, [lane][row] so that a lane's rows are
// adjacent: 32-bit cells keep K/2 bytes per row, cell k in byte k/2 at bit
// 4 (k & 1); 16-bit cells keep K bytes per row for the group's two pairs,
// cell k in 32-bit word k/4, pair h in half h, at bit 4 (3 - (k & 3)).
constexpr uint32_t kOpEq = 7, kOpX = 8, kOpI = 1, kOpD = 2;   // BAM codes

// Walk the codes back from the pair's last cell (its answer's end) to its
// first (the start) and write the CIGAR runs in alignment order.  Runs on
// one lane per group.  Within the span every optimal local path begins at
// the start with positive prefix scores, so along the path the local
// recurrence (0 floor, E and F clamped at 0) makes the same choices as the
// anchored one the oracle runs.  key: the group's best cell, which must be
// the span's last cell with the pair's score.
template <int K, bool PKD>
__device__ void trace_walk(const KParams &P, const PairRef &pr, uint64_t key,
                           const uint8_t *codes, bool fits, int W, int half, int rows,
                           BaseStream qs, BaseStream ts) {
    if (pr.id < 0) return;
    const int64_t p = pr.id;
    const int32_t want = P.in_score[p];
    auto fail = [&](int32_t code) {
        P.cig_len[p] = code;
        atomicAdd(P.errors, 1ull);
    };
    if (pr.invalid) return fail(-1);
    if (want <= 0) {
        P.cig_len[p] = 0;
        return;
    }
    if (!fits) return fail(-2);
    const int32_t s = (int32_t)(key >> 32);
    const int32_t col = (int32_t)(0xFFFFu - (uint32_t)(key & 0xFFFF));
    const int32_t row = (int32_t)(0xFFFFu - (uint32_t)((key >> 16) & 0xFFFF));
    if (s != want || row != pr.n - 1 || col != pr.m - 1) return fail(-1);
    const int64_t base = P.cig_off[p];
    const int64_t cap = P.cig_off[p + 1] - base;
    uint32_t *out = P.cig + base;
    // W and K are powers of two: column j is in chunk j >> log2(W K), lane
    // (j >> log2 K) & (W - 1), slot j & (K - 1); a 32-bit word holds 4
    // cells of a row (16-bit cells, this pair's half) or 8 (32-bit cells)
    const int lw = __builtin_ctz((unsigned)W), lk = __builtin_ctz((unsigned)K);
    constexpr int kPerWord = PKD ? 4 : 8;
    auto word_at = [&](int r, int c) -> uint32_t {
        const int ch = c >> (lw + lk), lq = (c >> lk) & (W - 1), k = c & (K - 1);
        const int64_t at = ((int64_t)ch * rows + r) * W + lq;
        return PKD ? reinterpret_cast<const uint32_t *>(codes + at * K)[k >> 2]
                   : reinterpret_cast<const uint32_t *>(codes + at * (K / 2))[k >> 3];
    };
    int i = pr.n - 1, j = pr.m - 1, state = 0;   // 0: H, 1: E, 2: F
    // the code word of cell (i, j), and the packed bases at q0 + j and t0 + i
    // with the words before them already requested (the walk goes up and
    // left, so a word's bases are used on consecutive steps)
    uint32_t cw = word_at(i, j);
    int64_t qp = pr.q0 + j, tp = pr.t0 + i;
    uint32_t qcur = qs.word(qp >> 4), qprv = qs.word((qp >> 4) - 1);
    uint32_t tcur = ts.word(tp >> 4), tprv = ts.word((tp >> 4) - 1);
    auto left = [&]() {
        if ((qp & 15) == 0) {
            qcur = qprv;
            qprv = qs.word((qp >> 4) - 2);
        }
        --qp;
        --j;
    };
    auto up = [&]() {
        if ((tp & 15) == 0) {
            tcur = tprv;
            tprv = ts.word((tp >> 4) - 2);
        }
        --tp;
        --i;
    };
    uint32_t run_op = 0, run_len = 0;
    int64_t nruns = 0;
    bool ok = true;
    // every op takes one step and every switch into a gap state another
    for (int64_t guard = 0; guard <= 2 * ((int64_t)pr.m + pr.n) + 4; ++guard) {
        if (i < 0 || j < 0) {
            ok = false;
            break;
        }
        const uint32_t nib = PKD ? (cw >> (16 * half + 4 * (3 - (j & 3)))) & 15u
                                 : (cw >> (4 * (j & 7))) & 15u;
        uint32_t op;
        bool done = false;
        if (state == 0) {
            // a gap state starts at this same cell: keep its word
            if (nib & 1u) {
                state = (nib & 2u) ? 2 : 1;
                continue;
            }
            const uint32_t qb = (qcur >> (2 * (qp & 15))) & 3u;
            const uint32_t tb = (tcur >> (2 * (tp & 15))) & 3u;
            op = qb == tb ? kOpEq : kOpX;
            done = i == 0 && j == 0;
            left();
            up();
            if (!done && i >= 0 && j >= 0) cw = word_at(i, j);
        } else if (state == 1) {
            op = kOpI;
            if (!((nib >> 2) & 1u)) state = 0;
            // the same word unless j was its first cell
            const bool same = (j & (kPerWord - 1)) != 0;
            left();
            if (!same && j >= 0) cw = word_at(i, j);
        } else {
            op = kOpD;
            if (!((nib >> 3) & 1u)) state = 0;
            up();
            if (i >= 0) cw = word_at(i, j);
        }
        if (op == run_op) {
            ++run_len;
        } else {
            if (run_len > 0) {
                if (nruns >= cap) { ok = false; break; }
                out[nruns++] = (run_len << 4) | run_op;
            }
            run_op = op;
            run_len = 1;
        }
        if (done) {
            if (nruns >= cap) { ok = false; break; }
            out[nruns++] = (run_len << 4) | run_op;
            run_len = 0;
            break;
        }
    }
    if (!ok || run_len != 0) return fail(-1);
    for (int64_t a = 0, b = nruns - 1; a < b; ++a, --b) {
        const uint32_t x = out[a];
        out[a] = out[b];
        out[b] = x;
    }
    P.cig_len[p] = (int32_t)nruns;
}

// Cell types of a unit: 32-bit integers (one pair per group), or two pairs
// per group in the 16-bit halves of every register, as saturating 16-bit
// integers or as binary16 numbers.
enum CellType : int { kCellWide = 0, kCellU16 = 1, kCellF16 = 2 };

// Strip split: one unit (a 64-lane group holding one or two long pairs) on
// several waves of a workgroup, for latency.  The target rows are cut into
// nw strips; wave ws runs every chunk of strip ws, in chunk order.  Chunk c
// of strip ws starts from the bottom row of chunk c of strip ws - 1 (H of
// its last row and F of the row after, per column: 2K words per lane),
// which that strip's wave stores when it finishes the chunk, into a ring
// of kSplitRing entries in its global slot; per-strip counters in LDS say
// how many chunks each strip has produced and taken.  A strip waits only
// for the strip above to produce and the strip below to take: the last
// strip never waits to produce and the first never waits for input, so
// every wait ends (each wait is also bounded: after kSpinLimit polls the
// unit is flagged and its pairs get -1).
constexpr int kSplitRing = 4;
constexpr int kSpinLimit = 1 << 22;
struct SplitCtx {
    int nw, ws;            // strips of the unit, this wave's strip
    int r_lo, r_hi;        // this strip's target rows
    uint32_t *ring;        // this wave's top-row ring (global, 2K words per lane per entry)
    uint32_t *ring_above;  // the ring of strip ws - 1
    int32_t *prod, *cons;  // LDS [nw]: chunks produced / taken by each strip
    int32_t *fail;         // LDS: set when a wait gave up
    unsigned long long *keys;  // LDS [nw][2]: each strip's best per pair
};
__device__ __forceinline__ bool wait_at_least(int32_t *p, int32_t v, int32_t *fail) {
    for (int it = 0; it < kSpinLimit; ++it) {
        const int32_t x = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
        if (x >= v) return true;
        if (__builtin_amdgcn_readfirstlane(
                __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return false;
}

// One unit: G = 64/W groups; each group aligns NPG pairs (2 packed, 1 wide).
// pos0: first position (in processing order) of the unit's pairs.
// [g0, g0 + gn): the groups processed in this pass (all G normally; fewer
// when the unit's boundary columns do not fit one slot together).
//
// BAND (SALoBa, Section VII-B: only cells near the main diagonal): cells
// with |i - j| > P.band do not exist.  A chunk of columns [c0, c0 + W*K)
// then only runs rows max(0, c0 - w) .. min(R-1, c0 + W*K - 1 + w); rows
// above that range are outside the band in every column of the chunk, so
// the zero column state stands for them exactly.  Every cell outside the
// band has its H forced to 0 before E, F and the row maximum read it: the
// band is contiguous in every row and column, so an out-of-band cell left
// of (below) the band only ever sees the boundary's E (F), and one right
// of (above) it only feeds other out-of-band cells -- with H = 0 the
// in-band cells see exactly the boundary values of the restricted table.
template <int K, int CT, bool REV, bool NM, bool BAND, bool TR, bool SPL = false>
__device__ __forceinline__ void run_unit(const KParams &P, BaseStream qs, BaseStream ts,
                                         BaseStream qm, BaseStream tm,
                         int64_t pos0, int64_t pos_end, int g0, int gn, int W,
                         uint32_t *slot, uint32_t *lds_saved, uint32_t *lds_bnd,
                         const SplitCtx *sp = nullptr) {
    const int G = kWave / W;
    constexpr bool PK = CT != kCellWide;
    constexpr int NPG = PK ? 2 : 1;
    static_assert(K % 4 == 0 && K <= 32, "K must be 4..32, multiple of 4");
    static_assert(!(BAND && (REV || NM)), "the banded pass is forward, without N masks");
    static_assert(!TR || (CT != kCellF16 && !REV && !NM && !BAND),
                  "the trace pass runs integer cells, forward, without masks or band");
    static_assert(!SPL || (CT != kCellWide && !REV && !NM && !BAND && !TR),
                  "the strip split runs the forward pass in 16-bit cells");
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / W;          // W is a power of two
    const int l = lane & (W - 1);
    const bool mine = g >= g0 && g < g0 + gn;

    PairRef pr[NPG];
#pragma unroll
    for (int h = 0; h < NPG; ++h)
        pr[h] = load_pair<REV, TR>(P, pos0 + (int64_t)g * NPG + h, pos_end, mine);

    int rmax = 0, mmax = 0;
#pragma unroll
    for (int h = 0; h < NPG; ++h) {
        rmax = max(rmax, pr[h].n);
        mmax = max(mmax, pr[h].m);
    }
    const int R = wave_max(rmax);
    // no target rows: every score is 0 and no boundary row may be touched
    const int Cw = wave_max((mmax + W * K - 1) / (W * K));
    int C = R > 0 ? Cw : 0;
    // banded: half-width w; a chunk starting past column R-1+w has no cell
    // in the band, nor does any chunk after it
    const int bw = BAND ? P.band : 0;
    if constexpr (BAND) {
        if (C > 0) C = min(C, (R - 1 + bw) / (W * K) + 1);
    }
    // boundary rows live at slot row (row & rwrap): a ring when banded
    uint32_t rwrap = 0xFFFFFFFFu;
    if constexpr (BAND) (void)band_slot_rows(R, bw, &rwrap);
    const int Gs = gn;           // groups sharing the slot, row-interleaved
    // slot column of this lane's group; lanes of groups outside this pass
    // still issue the (unused) boundary prefetch, so they read column 0
    const int gs = mine ? g - g0 : 0;

    Best best[NPG];
#pragma unroll
    for (int h = 0; h < NPG; ++h) best[h] = Best{0, -1, -1};

    // scoring constants
    const int32_t a = P.match, b = P.mismatch;
    const int32_t alpha = P.gap_open + P.gap_extend, beta = P.gap_extend;
    const uint32_t KC = (uint32_t)(a - b);               // byte: match - mismatch
    const uint32_t NB2 = (uint32_t)(-b) * 0x10001u;
    const uint32_t AL2 = (uint32_t)alpha * 0x10001u;
    const uint32_t BE2 = (uint32_t)beta * 0x10001u;
    // binary16 cells: -alpha and -beta in both halves; the row table holds
    // the high byte of match or mismatch as binary16 (their low bytes are 0)
    const uint32_t hm = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)a) >> 8;
    const uint32_t hx = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)b) >> 8;
    const uint32_t MM4 = hx * 0x01010101u;       // every base a mismatch
    const uint32_t XM = hm ^ hx;                 // flips one slot to match
    const uint32_t NAL2 =
        (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(-alpha)) * 0x10001u;
    const uint32_t NBE2 =
        (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)(-beta)) * 0x10001u;

    uint32_t *my_saved = lds_saved + (size_t)lane * (2 * K);
    // (strip split: the column in the slot's lower half, the top-row ring in
    // its upper half)
    const Slot bslot{slot, (uint32_t)P.slot_words * (SPL ? 2u : 4u)};
    // trace pass: this group's share of the block's code slot; the pair's
    // codes take (its chunks) x n rows x W lanes x K/2 bytes, laid out
    // [chunk][row][lane] so that the group's stores of one step are
    // adjacent and fill whole lines quickly (16-bit cells: the group's two
    // pairs share K bytes per lane and row, over the larger pair's chunks
    // and rows)
    uint8_t *tr_codes = nullptr;
    uint8_t *tr_wave = nullptr;    // the wave's code slot (at most 1 GiB)
    uint32_t tr_goff = 0;          // this group's share in it
    bool tr_fits = false;
    int tr_chunks = 0, tr_rows = 0;
    constexpr int kTrRowBytes = PK ? K : K / 2;
    const int tr_stride = W * kTrRowBytes;   // bytes from one row to the next
    if constexpr (TR) {
        const int64_t gslot = (P.trace_slot / G) & ~(int64_t)15;
        int mg = 0;
#pragma unroll
        for (int h = 0; h < NPG; ++h) {
            mg = max(mg, pr[h].m);
            tr_rows = max(tr_rows, pr[h].n);
        }
        tr_chunks = (mg + W * K - 1) / (W * K);
        tr_fits = (int64_t)tr_chunks * W * tr_rows * kTrRowBytes <= gslot;
        tr_wave = P.trace_ws + (int64_t)blockIdx.x * P.trace_slot;
        tr_goff = (uint32_t)(g * gslot);
        tr_codes = tr_wave + tr_goff;
    }
    // slot byte offsets: row r of this lane's group is at (r & rwrap) *
    // row_bytes + ld_lane; a row past the rows the previous chunk wrote
    // reads as 0 through the descriptor's range check (rows below 64 Ki and
    // at most 64 groups keep every offset in 32 bits)
    const uint32_t row_bytes = (uint32_t)Gs * 8u;
    const uint32_t ld_lane = (uint32_t)gs * 8u;
    // strip split: this wave's target rows [v_lo, v_lo + rows); rows outside
    // them (and past each pair's end) get the zero substitution table
    const int v_lo = SPL ? sp->r_lo : 0;
    const int Rc = SPL ? sp->r_hi - sp->r_lo : R;     // rows of the boundary column
    int lim[NPG];
#pragma unroll
    for (int h = 0; h < NPG; ++h)
        lim[h] = SPL ? max(0, min(pr[h].n, sp->r_hi) - v_lo) : pr[h].n;
    // the fewest rows of any pair of this pass's groups (the lanes of other
    // groups compute values nothing reads)
    int lim_min = 0x7FFFFFFF;
#pragma unroll
    for (int h = 0; h < NPG; ++h) lim_min = mine ? min(lim_min, lim[h]) : lim_min;
    lim_min = wave_min_i32(lim_min);
    // unbanded: the column in LDS, resident when the whole column fits, else
    // through the rings (Gs is then a power of two, so a 1 KiB block holds
    // SB = 128 / Gs whole rows)
    const bool bnd_res = (uint32_t)Rc * row_bytes <= kBndLdsBytes;
    const uint32_t bnd_mask = bnd_res ? 0xFFFFFFFFu : 2u * kBndBlockBytes - 1u;
    const uint32_t bnd_wbase = bnd_res ? 0u : 2u * kBndBlockBytes;
    const int sb_shift = __builtin_ctz(kBndBlockBytes / row_bytes);
    const uint32_t lane16 = (uint32_t)lane * 16u;

    for (int c = 0; c < C; ++c) {
        const int col0 = c * W * K + l * K;
        const int c0 = c * W * K;
        // rows of this chunk: r0 .. r0 + nrows - 1 (all rows unbanded);
        // step s runs row r0 + s - l on lane l
        const int r0 = BAND ? max(0, c0 - bw) : v_lo;
        const int nrows = BAND ? min(R - 1, c0 + W * K - 1 + bw) - r0 + 1 : Rc;
        // last row the previous chunk wrote to the slot
        const int bnd_hi = BAND ? min(R - 1, c0 - 1 + bw) : R - 1;
        auto slot_off = [&](int row) -> uint32_t {
            return row <= bnd_hi ? ld_lane + ((uint32_t)row & rwrap) * row_bytes
                                 : bslot.bytes;
        };
        // per-lane target stream geometry (per pair of the group)
        int64_t twi[NPG];
        uint32_t tsh[NPG];
#pragma unroll
        for (int h = 0; h < NPG; ++h) {
            // forward: lane l reads row r0 + s - l at base t0 + r0 + s - l,
            // 16 rows per word starting at t0 + r0 - l; REV: base
            // t0 - (s - l), so each 16-row word is the 16 bases ending at
            // t0 + l - s0, reversed, and the word index steps down
            const int64_t p0 = REV ? pr[h].t0 + l - 15 : pr[h].t0 + r0 - l;
            twi[h] = p0 >> 4;                    // floor for negatives
            tsh[h] = (uint32_t)(p0 & 15) * 2u;
        }
        // query selectors (PK) or query bases (wide) of this lane's K columns
        uint32_t SEL[K];
        {
            // this lane's query bases as up to two 16-base words per pair
            constexpr int NQW = (K + 15) / 16;
            uint32_t qw[NPG][NQW];
            // NM: N bits of the lane's columns (bit k = column col0 + k)
            uint32_t qn[NPG];
#pragma unroll
            for (int h = 0; h < NPG; ++h) {
                qn[h] = 0u;
                if constexpr (NM) {
                    if constexpr (REV)
                        qn[h] = __builtin_bitreverse32(qm.bits32(pr[h].q0 - col0 - 31));
                    else
                        qn[h] = qm.bits32(pr[h].q0 + col0);
                }
            }
#pragma unroll
            for (int h = 0; h < NPG; ++h) {
                // REV: column col0 + k is base q0 - col0 - k, so read the
                // 16*NQW bases ending at q0 - col0 and reverse them
                const int64_t p0 = REV ? pr[h].q0 - col0 - (16 * NQW - 1) : pr[h].q0 + col0;
                const uint32_t sh = (uint32_t)(p0 & 15) * 2u;
                uint32_t prev = qs.word(p0 >> 4);
#pragma unroll
                for (int w = 0; w < NQW; ++w) {
                    const uint32_t next = qs.word((p0 >> 4) + 1 + w);
                    qw[h][w] = __builtin_amdgcn_alignbit(next, prev, sh);
                    prev = next;
                }
                if constexpr (REV) {
                    if constexpr (NQW == 1) {
                        qw[h][0] = rev2(qw[h][0]);
                    } else {
                        const uint32_t w0 = qw[h][0];
                        qw[h][0] = rev2(qw[h][1]);
                        qw[h][1] = rev2(w0);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if constexpr (PK) {
                    // a column past the query's end, or an N, selects 0:
                    // a mismatch in 16-bit integers (binary16 never has N)
                    const uint32_t sA = (col0 + k < pr[0].m && !((qn[0] >> k) & 1u))
                                            ? ((qw[0][k >> 4] >> (2 * (k & 15))) & 3u) : 12u;
                    const uint32_t sB = (col0 + k < pr[1].m && !((qn[1] >> k) & 1u))
                                            ? (4u + ((qw[1][k >> 4] >> (2 * (k & 15))) & 3u)) : 12u;
                    // 16-bit integers: table byte low, 0 high; binary16:
                    // 0 low, table byte high (a column past the query's end
                    // selects 0 in both bytes)
                    if constexpr (CT == kCellU16)
                        SEL[k] = sA | (sB << 16) | 0x0C000C00u;
                    else
                        SEL[k] = (sA << 8) | (sB << 24) | 0x000C000Cu;
                } else {
                    SEL[k] = (col0 + k < pr[0].m && !((qn[0] >> k) & 1u))
                                 ? ((qw[0][k >> 4] >> (2 * (k & 15))) & 3u) : 5u;
                }
            }
        }

        // per column: H of the last row (the next row's diagonal) and F of
        // the next row, F(i+1,j) = max(F(i,j) - beta, H(i,j) - alpha)
        uint32_t H[K], F[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            H[k] = 0;
            F[k] = 0;
        }
        uint32_t hprev = 0;           // H(i-1, col0-1)
        // trace pass: whether F of the next row's columns extends (F(i+1, j)
        // != H(i, j) - alpha) -- 32-bit cells: bit k; 16-bit cells: bit 0 of
        // each cell's nibble, in the code words' layout -- and where this
        // lane's codes of the chunk go
        uint32_t fbits = 0;
        uint32_t facc[TR && PK ? K / 4 : 1];
#pragma unroll
        for (int w = 0; w < (TR && PK ? K / 4 : 1); ++w) facc[w] = 0;
        // 16-bit trace codes: the packed constants 1, 2, 4 and 16
        const uint32_t C1 = TR && PK ? opaque(0x00010001u) : 0u;
        const uint32_t C2 = TR && PK ? opaque(0x00020002u) : 0u;
        const uint32_t C4 = TR && PK ? opaque(0x00040004u) : 0u;
        const uint32_t C16 = TR && PK ? opaque(0x00100010u) : 0u;
        // 16-bit cells at 16 columns: a lane's codes of a row are 16 bytes,
        // and lanes 2k and 2k+1 of one row share a 32-byte sector.  Lane 2k
        // reaches the row a step before lane 2k+1, so it holds its codes for
        // one step and the two halves of each sector are stored together.
        constexpr bool TR_PAIRED = TR && PK && K == 16;
        uint32_t tr_held[TR_PAIRED ? 4 : 1];
#pragma unroll
        for (int w = 0; w < (TR_PAIRED ? 4 : 1); ++w) tr_held[w] = 0;
        const bool tr_delay = TR_PAIRED && W > 1 && (l & 1) == 0;
        const uint32_t tr_dmask = tr_delay ? ~0u : 0u;
        // the row a lane stores at step s is i - delay = r0 + s - l - delay,
        // at tr_wave + tr_goff + (chunk, lane offset) + row * tr_stride: a
        // wave-uniform part that moves with s, and a 32-bit lane part made
        // non-negative by W + 1 rows taken from the uniform part
        bool tr_on = false;
        uint32_t tr_loff = 0;
        if constexpr (TR) {
            tr_on = tr_fits && mine && c < tr_chunks;
            tr_loff = tr_goff + ((uint32_t)c * (uint32_t)tr_rows * (uint32_t)W + (uint32_t)l) *
                                    (uint32_t)kTrRowBytes +
                      (uint32_t)(r0 - l - (tr_delay ? 1 : 0) + W + 1) * (uint32_t)tr_stride;
        }
        auto tr_dst = [&](int s) -> uint8_t * {
            return tr_wave + (int64_t)(s - W - 1) * tr_stride + tr_loff;
        };
        uint32_t hout = 0, eout = 0;  // outputs of this lane's last processed row
        uint32_t cbest = 0;           // packed (or wide) best row maximum in this chunk
        int32_t crow[NPG];
#pragma unroll
        for (int h = 0; h < NPG; ++h) crow[h] = -1;
        // 16-bit cells: which of the lane's two row buffers holds each pair's
        // saved row, one bit per lane of the wave (set: buffer 1); a row where
        // both pairs improve is saved once for both
        uint64_t sbA = 0ull, sbB = ~0ull;

        const bool have_bnd = c > 0;   // implies R >= 1 (C == 0 when R == 0)
        const bool write_bnd = c + 1 < C;
        const bool first_lane = l == 0;
        const bool last_lane = l == W - 1 && mine;
        constexpr int kRowWords = kWave * 2 * K;   // one ring entry: 2K words per lane
        if constexpr (SPL) {
            // this chunk's bottom row goes to ring entry c mod kSplitRing:
            // wait until the strip below has taken the chunk that used it
            if (sp->ws + 1 < sp->nw && c >= kSplitRing)
                (void)wait_at_least(sp->cons + sp->ws + 1, c - kSplitRing + 1, sp->fail);
            if (sp->ws > 0) {
                // start from this chunk's bottom row in the strip above: H of
                // row r_lo - 1 and F of row r_lo per column; lane 0's diagonal
                // is H of row r_lo - 1 in the previous chunk's last column
                if (wait_at_least(sp->prod + sp->ws - 1, c + 1, sp->fail)) {
                    const uint32_t *e = sp->ring_above + (size_t)(c % kSplitRing) * kRowWords +
                                        (size_t)lane * (2 * K);
#pragma unroll
                    for (int k = 0; k < K; k += 4) {
                        const uint4 hv = *reinterpret_cast<const uint4 *>(e + k);
                        const uint4 fv = *reinterpret_cast<const uint4 *>(e + K + k);
                        H[k] = hv.x; H[k + 1] = hv.y; H[k + 2] = hv.z; H[k + 3] = hv.w;
                        F[k] = fv.x; F[k + 1] = fv.y; F[k + 2] = fv.z; F[k + 3] = fv.w;
                    }
                    const uint32_t d0 =
                        c > 0 ? sp->ring_above[(size_t)((c - 1) % kSplitRing) * kRowWords +
                                               (size_t)(kWave - 1) * (2 * K) + (K - 1)]
                              : 0u;
                    hprev = shift_in(H[K - 1], d0, first_lane);
                    // the entry may be reused once these loads are done
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                }
                if (lane == 0)
                    __hip_atomic_store(sp->cons + sp->ws, c + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        // banded: the boundary rows of the next four steps, in flight
        uint2 fifo[BAND ? 4 : 1];
        // unbanded: the boundary row of the current step (read one step
        // ahead from LDS) and, in ring mode, the next block in flight
        uint2 bnd_cur = make_uint2(0u, 0u);
        uint4 inflight = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (BAND) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                fifo[r] = make_uint2(0u, 0u);
                if (have_bnd) fifo[r] = bslot.load(slot_off(r0 + r));
            }
        } else {
            if (have_bnd) {
                if (!bnd_res) {
                    // blocks 0 and 1 into the read ring, then block 2 in flight
                    const uint4 b0 = bslot.load16(lane16);
                    const uint4 b1 = bslot.load16(kBndBlockBytes + lane16);
                    lds_store16(lds_bnd, lane16, b0);
                    lds_store16(lds_bnd, kBndBlockBytes + lane16, b1);
                    wave_sync();
                    inflight = bslot.load16(2u * kBndBlockBytes + lane16);
                }
            } else {
                // the first chunk has no boundary: it reads zeros from the
                // column (resident) or from the read ring, which no block
                // event refills during this chunk
                const uint4 z = make_uint4(0u, 0u, 0u, 0u);
                lds_store16(lds_bnd, lane16, z);
                lds_store16(lds_bnd, kBndBlockBytes + lane16, z);
                if (bnd_res) {
                    lds_store16(lds_bnd, 2u * kBndBlockBytes + lane16, z);
                    lds_store16(lds_bnd, 3u * kBndBlockBytes + lane16, z);
                }
                wave_sync();
            }
            bnd_cur = lds_load8(lds_bnd, ld_lane);      // row 0
        }
        if constexpr (BAND) {
            // lane 0's first diagonal: H(r0 - 1, c0 - 1), inside the band
            if (have_bnd && r0 > 0) {
                const uint32_t hd0 = bslot.load(slot_off(r0 - 1)).x;
                hprev = first_lane ? hd0 : 0u;
            }
        }
        // banded: i - col0 at step 0; the lane's in-band columns at step s
        // are k in [dl + s - w, dl + s + w]
        const int dl = r0 - c0 - l * (K + 1);
        // lane l covers all its columns at step s when dl + s - w <= 0 and
        // dl + s + w >= K - 1: for every lane exactly when s_lo <= s <= s_hi
        const int s_hi = bw - (r0 - c0);
        const int s_lo = K - 1 + (W - 1) * (K + 1) - bw - (r0 - c0);

        const int S = nrows + W - 1;
        uint32_t tw_lo[NPG], tw_hi[NPG];
#pragma unroll
        for (int h = 0; h < NPG; ++h) {
            tw_lo[h] = ts.word(twi[h]);
            tw_hi[h] = ts.word(twi[h] + 1);
        }
        uint32_t tw[NPG];
#pragma unroll
        for (int h = 0; h < NPG; ++h) tw[h] = 0;
        // NM: N bits of the 16 target rows of the current word (bit j = row
        // s0 + j - l of this lane), and of the next 16, in flight
        uint32_t tn[NPG], tn_nx[NPG];
        auto target_n_bits = [&](int h, int s0w) -> uint32_t {
            if constexpr (REV)
                return __builtin_bitreverse32(tm.bits32(pr[h].t0 + l - 15 - s0w)) >> 16;
            else
                return tm.bits32(pr[h].t0 - l + s0w);
        };
#pragma unroll
        for (int h = 0; h < NPG; ++h) {
            tn[h] = 0u;
            tn_nx[h] = 0u;
            if constexpr (NM) tn_nx[h] = target_n_bits(h, 0);
        }
        // steps s0 .. s0+3 for s0 = sa, sa+4, ... < sb (sa a multiple of 4)
        // `frozen` (compile time): strip split, the first W - 1 steps of a
        // strip below the first, where lane l has no row before step l and
        // keeps its starting state
        // `bulk` (compile time, unbanded): every step of the range has
        // s >= W - 1 and s + 1 < Rc, so the step-range checks of the
        // boundary reader and writer are left out
        auto run_steps = [&](int sa, int sb, auto masked, auto frozen, auto bulk,
                             auto full) {
        for (int s0 = sa; s0 < sb; s0 += 4) {
            if ((s0 & 15) == 0) {
                // the next 16 target bases of each pair, already in flight;
                // start loading the 16 after them
#pragma unroll
                for (int h = 0; h < NPG; ++h) {
                    tw[h] = __builtin_amdgcn_alignbit(tw_hi[h], tw_lo[h], tsh[h]);
                    if constexpr (REV) tw[h] = rev2(tw[h]);
                    const int64_t wi = REV ? twi[h] - ((s0 + 16) >> 4) : twi[h] + ((s0 + 16) >> 4);
                    tw_lo[h] = ts.word(wi);
                    tw_hi[h] = ts.word(wi + 1);
                    if constexpr (NM) {
                        tn[h] = tn_nx[h];
                        tn_nx[h] = target_n_bits(h, s0 + 16);
                    }
                }
            }
            const uint32_t jsh = (uint32_t)(s0 & 15) * 2u;
            // four steps; `masked` (compile time) applies the band mask
            auto steps4 = [&](auto masked) {
            constexpr bool MASK = BAND && decltype(masked)::value;
            constexpr bool FROZEN = SPL && decltype(frozen)::value;
            constexpr bool BULK = !BAND && decltype(bulk)::value;
            // every row of every lane lies below each of its pairs' ends
            // (and at or above row 0): no per-pair range test
            constexpr bool FULL = BULK && !NM && decltype(full)::value;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int s = s0 + j;
                if (BULK || s < S) {
                const int i = r0 + s - l;
                uint2 bnd;
                if constexpr (BAND) {
                    bnd = fifo[j & 3];
                    if (have_bnd) fifo[j & 3] = bslot.load(slot_off(r0 + s + 4));
                } else {
                    bnd = bnd_cur;
                    // row rn = s + 1 for the next step (rows past the column
                    // read as 0); in ring mode its block is in the read ring
                    // (see the block events below); the first chunk reads
                    // the zeros its start cleared
                    const int rn = s + 1;
                    bnd_cur = (BULK || rn < Rc)
                                  ? lds_load8(lds_bnd,
                                              (((uint32_t)rn * row_bytes) & bnd_mask) + ld_lane)
                                  : make_uint2(0u, 0u);
                }
                // banded: bit k set when column col0 + k of row i is in the band
                uint32_t bmask = 0xFFFFFFFFu;
                if constexpr (MASK) {
                    const int lo = max(dl + s - bw, 0);
                    const int hi = min(dl + s + bw + 1, K);
                    bmask = hi > lo ? (0xFFFFFFFFu >> (32 - (hi - lo))) << lo : 0u;
                }
                // all ones, or 0 for a column outside the band
                auto inband = [&](int k) -> uint32_t {
                    return MASK ? (uint32_t)((int32_t)(bmask << (31 - k)) >> 31) : 0xFFFFFFFFu;
                };
                // packed cells: this row's maxima of a live lane (0 otherwise),
                // for the first-maximum tracking after the lane's step
                uint32_t rowmax_live = 0;
                if (!FROZEN || l <= s) {
                const uint32_t hin = shift_in(hout, bnd.x, first_lane);
                const uint32_t ein = shift_in(eout, bnd.y, first_lane);
                // every lane runs every step: rows outside [0, n) of a pair
                // (the wavefront ramp, and rows past the shorter pairs of the
                // unit) use a zero substitution table, so each of their
                // values is bounded by a real cell of an earlier row and can
                // never become, or tie ahead of, the first maximum
                uint32_t e = ein;
                uint32_t hd = hprev;
                uint32_t rowmax = 0;
                if constexpr (CT == kCellF16) {
                    // S(i,j) = hd + table value, as binary16 numbers;
                    // E is clamped at 0 (so H >= 0 needs no fourth
                    // operand); F may go negative, down to -alpha
                    const uint32_t bA = (tw[0] >> (jsh + 2 * j)) & 3u;
                    const uint32_t bB = (tw[1] >> (jsh + 2 * j)) & 3u;
                    const uint32_t TA = (FULL || (uint32_t)(i - v_lo) < (uint32_t)lim[0])
                                            ? (MM4 ^ (XM << (bA << 3))) : 0u;
                    const uint32_t TB = (FULL || (uint32_t)(i - v_lo) < (uint32_t)lim[1])
                                            ? (MM4 ^ (XM << (bB << 3))) : 0u;
                    // the diagonal term of column k+1 is formed in column
                    // k's step, from H[k] before it takes row i: it is
                    // independent of the E chain (hh, ha, e), so it fills
                    // the gap gfx950 needs between two packed instructions
                    // when the second reads the first's result
                    uint32_t dk = hadd(hd, __builtin_amdgcn_perm(TB, TA, SEL[0]));
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t dnext =
                            k + 1 < K ? hadd(H[k], __builtin_amdgcn_perm(TB, TA, SEL[k + 1]))
                                      : 0u;
                        const uint32_t f = F[k];
                        const uint32_t hh = pmax3(dk, f, e) & inband(k);
                        dk = dnext;
                        H[k] = hh;
                        const uint32_t ha = hadd(hh, NAL2);
                        F[k] = hmax(hadd(f, NBE2), ha);
                        e = pmax3(hadd(e, NBE2), ha, 0u);
                        if (k & 1)
                            rowmax = k == 1 ? pmax(H[0], hh) : pmax3(rowmax, H[k - 1], hh);
                    }
                } else if constexpr (CT == kCellU16) {
                    const uint32_t bA = (tw[0] >> (jsh + 2 * j)) & 3u;
                    const uint32_t bB = (tw[1] >> (jsh + 2 * j)) & 3u;
                    // rows past the pair's end (and N rows) get the zero
                    // table: a mismatch in every column
                    bool okA = FULL || (uint32_t)(i - v_lo) < (uint32_t)lim[0];
                    bool okB = FULL || (uint32_t)(i - v_lo) < (uint32_t)lim[1];
                    if constexpr (NM) {
                        okA = okA && !((tn[0] >> ((s0 & 15) + j)) & 1u);
                        okB = okB && !((tn[1] >> ((s0 & 15) + j)) & 1u);
                    }
                    const uint32_t TA = okA ? (KC << (bA << 3)) : 0u;
                    const uint32_t TB = okB ? (KC << (bB << 3)) : 0u;
                    // diagonal term of column k+1 formed in column k's
                    // step, as in the binary16 loop
                    uint32_t dk = psub(padd(hd, __builtin_amdgcn_perm(TB, TA, SEL[0])), NB2);
                    // trace pass: code words of this row, and the F bits
                    // for the next one (each word starts at its first cell)
                    uint32_t acc[TR ? K / 4 : 1] = {}, fnew[TR ? K / 4 : 1] = {};
                    uint32_t ha_left = 0;          // H(i, j-1) - alpha
                    if constexpr (TR) ha_left = psub(hin, AL2);
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t dnext =
                            k + 1 < K ? psub(padd(H[k], __builtin_amdgcn_perm(TB, TA, SEL[k + 1])),
                                             NB2)
                                      : 0u;
                        const uint32_t f = F[k];
                        const uint32_t hh = pmax3(dk, f, e) & inband(k);
                        if constexpr (TR) {
                            // H >= the diagonal term and >= E; E >= H(i, j-1) - alpha
                            const uint32_t nd = pnz(psub(hh, dk), C1);
                            const uint32_t ne = pnz(psub(hh, e), C1);
                            const uint32_t ex = pnz(psub(e, ha_left), C1);
                            const uint32_t nib = sealed(pmad(ex, C4, pmad(ne, C2, nd)));
                            acc[k >> 2] = (k & 3) ? pmad(acc[k >> 2], C16, nib) : nib;
                        }
                        dk = dnext;
                        H[k] = hh;
                        const uint32_t ha = psub(hh, AL2);
                        F[k] = pmax(psub(f, BE2), ha);
                        if constexpr (TR) {
                            // F(i+1, j) >= H(i, j) - alpha
                            const uint32_t fx = pnz(psub(F[k], ha), C1);
                            fnew[k >> 2] = (k & 3) ? pmad(fnew[k >> 2], C16, fx) : fx;
                            ha_left = ha;
                        }
                        e = pmax(psub(e, BE2), ha);
                        // row maximum two columns at a time
                        if (k & 1)
                            rowmax = k == 1 ? pmax(H[0], hh) : pmax3(rowmax, H[k - 1], hh);
                    }
                    if constexpr (TR) {
#pragma unroll
                        for (int w = 0; w < K / 4; ++w) {
                            acc[w] |= facc[w] << 3;    // bit 0 of each nibble to bit 3
                            facc[w] = fnew[w];
                        }
                        if constexpr (TR_PAIRED) {
                            // even lanes store the row before this one (held
                            // since the last step), odd lanes this row
                            const int row = tr_delay ? i - 1 : i;
                            const uint4 v = make_uint4(
                                (tr_held[0] & tr_dmask) | (acc[0] & ~tr_dmask),
                                (tr_held[1] & tr_dmask) | (acc[1] & ~tr_dmask),
                                (tr_held[2] & tr_dmask) | (acc[2] & ~tr_dmask),
                                (tr_held[3] & tr_dmask) | (acc[3] & ~tr_dmask));
                            if (tr_on && (uint32_t)row < (uint32_t)tr_rows)
                                *reinterpret_cast<uint4 *>(tr_dst(s)) = v;
#pragma unroll
                            for (int w = 0; w < 4; ++w) tr_held[w] = acc[w];
                        } else if (tr_on && (uint32_t)i < (uint32_t)tr_rows) {
                            uint8_t *dst = tr_dst(s);
                            if constexpr (K == 8) {
                                *reinterpret_cast<uint2 *>(dst) = make_uint2(acc[0], acc[1]);
                            } else {
                                *reinterpret_cast<uint4 *>(dst) =
                                    make_uint4(acc[0], acc[1], acc[2], acc[3]);
                            }
                        }
                    }
                } else {
                    bool okt = FULL || (uint32_t)(i - v_lo) < (uint32_t)lim[0];
                    if constexpr (NM) okt = okt && !((tn[0] >> ((s0 & 15) + j)) & 1u);
                    // 4 never equals a query code (0..3, or 5 past the end / N)
                    const uint32_t tb = okt ? ((tw[0] >> (jsh + 2 * j)) & 3u) : 4u;
#pragma unroll
                    for (int k = K - 1; k >= 0; --k)
                        H[k] = (uint32_t)((int)(k > 0 ? H[k - 1] : hd) +
                                          (SEL[k] == tb ? a : b));
                    uint32_t code[TR ? K / 8 : 1];
                    uint32_t fnext = 0;
#pragma unroll
                    for (int w = 0; w < (TR ? K / 8 : 1); ++w) code[w] = 0;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const int f = (int)F[k];
                        const int dv = (int)H[k];
                        const int hh = max3i(dv, f, (int)e) & (int)inband(k);
                        if constexpr (TR) {
                            // H(i, j-1): this row's value of the column to the left
                            const int hl = k > 0 ? (int)H[k - 1] : (int)hin;
                            uint32_t nib = hh != dv ? 1u : 0u;
                            nib |= hh != (int)e ? 2u : 0u;
                            nib |= (int)e != hl - alpha ? 4u : 0u;
                            nib |= ((fbits >> k) & 1u) << 3;
                            code[k >> 3] |= nib << (4 * (k & 7));
                        }
                        H[k] = (uint32_t)hh;
                        const int ha = hh - alpha;
                        F[k] = (uint32_t)max3i(f - beta, ha, 0);
                        if constexpr (TR) fnext |= ((int)F[k] != ha ? 1u : 0u) << k;
                        rowmax = k == 0 ? (uint32_t)hh : (uint32_t)max((int)rowmax, hh);
                        e = (uint32_t)max3i((int)e - beta, ha, 0);
                    }
                    if constexpr (TR) {
                        fbits = fnext;
                        if (tr_on && (uint32_t)i < (uint32_t)tr_rows) {
                            uint8_t *dst = tr_dst(s);
                            if constexpr (K == 8) {
                                *reinterpret_cast<uint32_t *>(dst) = code[0];
                            } else if constexpr (K == 16) {
                                *reinterpret_cast<uint2 *>(dst) = make_uint2(code[0], code[1]);
                            } else {
                                *reinterpret_cast<uint4 *>(dst) =
                                    make_uint4(code[0], code[1], code[2], code[3]);
                            }
                        }
                    }
                }
                if constexpr (CT != kCellWide) {
                    // keep the F updates in this block, among the E chain's
                    // independent work, rather than sunk below the row save
                    // where each add and max pair would stall
#pragma unroll
                    for (int k = 0; k < K; ++k) asm volatile("" ::"v"(F[k]));
                }
                hprev = hin;
                hout = H[K - 1];
                eout = e;
                if constexpr (SPL) {
                    // the strip's last row: the next strip starts from it
                    if (i == sp->r_hi - 1 && sp->ws + 1 < sp->nw) {
                        uint32_t *e2 = sp->ring + (size_t)(c % kSplitRing) * kRowWords +
                                       (size_t)lane * (2 * K);
#pragma unroll
                        for (int k = 0; k < K; k += 4) {
                            *reinterpret_cast<uint4 *>(e2 + k) =
                                make_uint4(H[k], H[k + 1], H[k + 2], H[k + 3]);
                            *reinterpret_cast<uint4 *>(e2 + K + k) =
                                make_uint4(F[k], F[k + 1], F[k + 2], F[k + 3]);
                        }
                    }
                }
                // row-level tracking of the first maximum (packed cells: after
                // the live-lane block, so that the wave-wide masks below are
                // formed in uniform control flow)
                if constexpr (PK) {
                    rowmax_live = rowmax;
                } else {
                    if ((int)rowmax > (int)cbest) {
                        cbest = rowmax;
                        crow[0] = i;
#pragma unroll
                        for (int k = 0; k < K; k += 4)
                            *reinterpret_cast<uint4 *>(my_saved + k) =
                                make_uint4(H[k], H[k + 1], H[k + 2], H[k + 3]);
                    }
                }
                }  // live lane
                if constexpr (PK) {
                    const uint32_t rowmax = rowmax_live;
                    // pair A in the low halves, pair B in the high halves;
                    // non-negative binary16 values order as their bits do
                    const bool cA = (rowmax & 0xFFFFu) > (cbest & 0xFFFFu);
                    const bool cB = (rowmax >> 16) > (cbest >> 16);
                    cbest = pmax(cbest, rowmax);
                    const uint64_t mA = __builtin_amdgcn_ballot_w64(cA);
                    const uint64_t mB = __builtin_amdgcn_ballot_w64(cB);
                    if ((mA | mB) != 0ull) {
                        // one save per row, the buffer chosen per lane with
                        // wave-wide masks: one pair improving alone takes the
                        // buffer the other pair's saved row is not in (the
                        // other buffer when both sit in one); both improving
                        // take pair A's
                        const uint64_t alone_eq = (mA ^ mB) & ~(sbA ^ sbB);
                        const uint64_t onlyB = mB & ~mA;
                        const uint64_t x = (alone_eq & ~sbA) |
                                           (~alone_eq & ((onlyB & sbB) | (~onlyB & sbA)));
                        sbA = (sbA & ~mA) | (x & mA);
                        sbB = (sbB & ~mB) | (x & mB);
                        if (cA) crow[0] = i;
                        if (cB) crow[1] = i;
                        if (cA || cB) {
                            uint32_t *dst =
                                my_saved + (__builtin_amdgcn_inverse_ballot_w64(x) ? K : 0);
#pragma unroll
                            for (int k = 0; k < K; k += 4)
                                *reinterpret_cast<uint4 *>(dst + k) =
                                    make_uint4(H[k], H[k + 1], H[k + 2], H[k + 3]);
                        }
                    }
                }
                // the group's last lane holds row r0 + s - (W-1): one of the
                // chunk's rows once s >= W-1 (and never past them, as
                // s < nrows + W - 1)
                if constexpr (BAND) {
                    if (write_bnd && s >= W - 1 && last_lane)
                        bslot.store(ld_lane + ((uint32_t)(r0 + s - (W - 1)) & rwrap) * row_bytes,
                                    hout, eout);
                } else if (write_bnd && (BULK || s >= W - 1)) {
                    // row r of this chunk's column into LDS; in ring mode a
                    // completed block goes to the slot as one burst
                    const uint32_t r = (uint32_t)(s - (W - 1));
                    if (last_lane)
                        lds_store8(lds_bnd, bnd_wbase + ((r * row_bytes) & bnd_mask) + ld_lane,
                                   hout, eout);
                }
                }  // s < S
            }
            if constexpr (!BAND) {
                // ring events of this block of four steps (a ring block
                // holds at least 4 rows, so at most one of each happens):
                //  * the rows written here completed block kw: the wave
                //    copies it to the slot as one burst;
                //  * the rows read here entered block kr: block kr + 1 (in
                //    flight) goes into the read ring in place of kr - 1,
                //    and kr + 2 is loaded (past the column it reads stale
                //    slot words or zeros; such rows are never used)
                if (!bnd_res) {
                    const int sh = sb_shift;
                    const int rw_hi = min(s0 + 3 - (W - 1), Rc - 1);
                    const int rw_lo = max(s0 - (W - 1), 0);
                    if (write_bnd && rw_hi >= rw_lo && ((rw_hi + 1) >> sh) > (rw_lo >> sh)) {
                        const uint32_t kw = (uint32_t)(((rw_hi + 1) >> sh) - 1);
                        asm volatile("" ::: "memory");
                        const uint4 v = lds_load16(lds_bnd, bnd_wbase +
                                                                (kw & 1u) * kBndBlockBytes + lane16);
                        bslot.store16(kw * kBndBlockBytes + lane16, v);
                    }
                    if (have_bnd && ((s0 + 4) >> sh) > (s0 >> sh)) {
                        const uint32_t kr = (uint32_t)((s0 + 4) >> sh);
                        lds_store16(lds_bnd, ((kr + 1u) & 1u) * kBndBlockBytes + lane16,
                                    inflight);
                        asm volatile("" ::: "memory");
                        inflight = bslot.load16((kr + 2u) * kBndBlockBytes + lane16);
                    }
                }
            }
            };
            steps4(masked);
        }
        };
        if constexpr (BAND) {
            // steps s_lo .. s_hi have every lane's K columns inside the band
            // (the same for every group of the wave): the 4-step blocks
            // inside that range skip the mask
            const int a = min(max(0, (s_lo + 3) & ~3), (S + 3) & ~3);
            const int b = max(a, min(((s_hi + 1) & ~3), (S + 3) & ~3));
            run_steps(0, a, std::true_type{}, std::false_type{}, std::false_type{}, std::false_type{});
            run_steps(a, b, std::false_type{}, std::false_type{}, std::false_type{}, std::false_type{});
            run_steps(b, S, std::true_type{}, std::false_type{}, std::false_type{}, std::false_type{});
        } else {
            // head (the wavefront's ramp: lanes before their first row; a
            // strip below the first keeps them frozen), bulk, tail (rows
            // past the column); the N-mask and trace kernels, which hold
            // more registers, keep one loop with the checks in every step
            // (bulk steps below `f` run every lane's row inside each of its
            // pairs, so they skip the per-pair range test)
            const int a = min((W - 1 + 3) & ~3, (S + 3) & ~3);
            const int b = max(a, (Rc - 1) & ~3);
            const int f = max(a, min(b, lim_min & ~3));
            if (SPL && sp->ws > 0) {
                run_steps(0, a, std::false_type{}, std::true_type{}, std::false_type{}, std::false_type{});
                run_steps(a, f, std::false_type{}, std::false_type{}, std::true_type{}, std::true_type{});
                run_steps(f, b, std::false_type{}, std::false_type{}, std::true_type{}, std::false_type{});
                run_steps(b, S, std::false_type{}, std::false_type{}, std::false_type{}, std::false_type{});
            } else if constexpr (!NM && !TR) {
                run_steps(0, a, std::false_type{}, std::false_type{}, std::false_type{}, std::false_type{});
                run_steps(a, f, std::false_type{}, std::false_type{}, std::true_type{}, std::true_type{});
                run_steps(f, b, std::false_type{}, std::false_type{}, std::true_type{}, std::false_type{});
                run_steps(b, S, std::false_type{}, std::false_type{}, std::false_type{}, std::false_type{});
            } else {
                run_steps(0, S, std::false_type{}, std::false_type{}, std::false_type{}, std::false_type{});
            }
        }
        if constexpr (TR_PAIRED) {
            // the even lanes' last row, still held
            const int row = r0 + S - 1 - l;
            if (tr_delay && tr_on && (uint32_t)row < (uint32_t)tr_rows)
                *reinterpret_cast<uint4 *>(tr_dst(S)) =
                    make_uint4(tr_held[0], tr_held[1], tr_held[2], tr_held[3]);
        }
        if constexpr (!BAND) {
            // ring mode: the column's last, partial block goes to the slot
            if (write_bnd && !bnd_res && ((uint32_t)Rc & ((1u << sb_shift) - 1u)) != 0) {
                asm volatile("" ::: "memory");
                const uint32_t kb = (uint32_t)Rc >> sb_shift;
                const uint4 v =
                    lds_load16(lds_bnd, bnd_wbase + (kb & 1u) * kBndBlockBytes + lane16);
                bslot.store16(kb * kBndBlockBytes + lane16, v);
            }
        }
        if constexpr (SPL) {
            // this chunk's bottom row is stored: the strip below may start it
            if (sp->ws + 1 < sp->nw) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if (lane == 0)
                    __hip_atomic_store(sp->prod + sp->ws, c + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }

        // resolve this chunk's candidate column per pair
#pragma unroll
        for (int h = 0; h < NPG; ++h) {
            const uint32_t v = PK ? ((cbest >> (16 * h)) & 0xFFFFu) : cbest;
            if ((int)v > 0) {
                int kk = K - 1;
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    const uint32_t hv =
                        PK ? ((my_saved[(__builtin_amdgcn_inverse_ballot_w64(h ? sbB : sbA)
                                             ? K : 0) + k] >> (16 * h)) & 0xFFFFu)
                           : my_saved[k];
                    if (hv == v) kk = k;
                }
                best[h].offer(CT == kCellF16 ? half_bits_to_int(v) : (int32_t)v, crow[h],
                              col0 + kk);
            }
        }
        // the slot's column becomes the next chunk's input: make the last
        // lanes' stores visible to lane 0 of every group
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }

    if constexpr (TR) {
        // one walker per pair: lane h of the group walks pair h, so the
        // group's two pairs walk at the same time (a one-lane group walks
        // them one after the other)
        uint64_t keys[NPG];
#pragma unroll
        for (int h = 0; h < NPG; ++h) keys[h] = group_max_u64(best[h].key(), W);
        if (W > 1) {
            if (mine && l < NPG) {
                const bool second = NPG > 1 && l == 1;
                trace_walk<K, PK>(P, second ? pr[NPG - 1] : pr[0],
                                  second ? keys[NPG - 1] : keys[0], tr_codes, tr_fits, W,
                                  second ? 1 : 0, tr_rows, qs, ts);
            }
        } else if (mine) {
#pragma unroll
            for (int h = 0; h < NPG; ++h)
                trace_walk<K, PK>(P, pr[h], keys[h], tr_codes, tr_fits, W, h, tr_rows, qs, ts);
        }
        return;
    }
#pragma unroll
    for (int h = 0; h < NPG; ++h) {
        const uint64_t key = group_max_u64(best[h].key(), W);
        if constexpr (SPL) {
            // the strips' bests merge in the workgroup (split_kernel)
            if (lane == 0) sp->keys[sp->ws * 2 + h] = key;
        } else {
            if (l == 0 && mine) {
                write_result<REV>(P, pr[h], key);
                if constexpr (!REV) signal_done(P, pr[h].id);
            }
        }
    }
}

// The narrowest cell type every pair of the unit admits.
template <bool REV>
__device__ __forceinline__ int unit_cell_type(const KParams &P, int64_t pos0, int npairs) {
    if (!P.packed_ok || P.force_int32) return kCellWide;
    const int lane = threadIdx.x & (kWave - 1);
    bool ok16 = true, okh = P.half_ok != 0;
    for (int k = lane; k < npairs; k += kWave) {
        const PairRef r = load_pair<REV>(P, pos0 + k, pos0 + npairs, true);
        if (r.id >= 0 && !r.invalid) {
            const int64_t mn = min(r.m, r.n);
            if (!packed_bound_ok(P.match, P.mismatch, mn)) ok16 = false;
            if (!half_bound_ok(P.match, mn)) okh = false;
        }
    }
    const bool all16 = __ballot(!ok16) == 0ull;
    const bool allh = __ballot(!okh) == 0ull;
    return __builtin_amdgcn_readfirstlane(all16 ? (allh ? kCellF16 : kCellU16) : kCellWide);
}

template <int K, bool REV, bool NM, bool BAND, bool TR>
__device__ __forceinline__ void process_unit(const KParams &P, BaseStream qs, BaseStream ts,
                                             BaseStream qm, BaseStream tm,
                                             int64_t pos0, int npairs, int W, uint32_t *slot,
                                             uint32_t *lds, uint32_t *lds_bnd) {
    const int G = kWave / W;
    // rows one slot holds for G groups; larger units run one group at a time
    int rmax = 0;
    const int lane = threadIdx.x & (kWave - 1);
    for (int k = lane; k < npairs; k += kWave) {
        const PairRef r = load_pair<REV, TR>(P, pos0 + k, pos0 + npairs, true);
        rmax = max(rmax, r.n);
    }
    const int R = wave_max(rmax);
    // slot rows per group: every target row, or the banded ring
    uint32_t wrap = 0;
    const int rows = BAND ? band_slot_rows(R, P.band, &wrap) : R;
    // groups whose boundary columns fit one slot together; a larger unit is
    // processed in several passes of that many groups.  One call site per
    // instantiation keeps run_unit inlined.
    int fit = (int)min<int64_t>(G, (int64_t)P.slot_words / (2 * (int64_t)max(rows, 1)));
    // unbanded passes keep a power-of-two group count (the LDS ring's
    // blocks hold whole rows); G is a power of two, so every pass is full.
    // A column that leaves LDS goes through 1 KiB ring blocks of at least
    // 4 rows, so at most 32 groups share it (1-lane groups then run in two
    // passes)
    if (!BAND) {
        fit = 1 << (31 - __builtin_clz((unsigned)fit));
        if (fit > 32 && (int64_t)rows * fit * 8 > (int64_t)kBndLdsBytes) fit = 32;
    }
    const int passes = (G + fit - 1) / fit;
    // with N masks the host turns binary16 cells off (their table cannot
    // give an N column the mismatch), so NM never instantiates them
    // the trace pass has binary16 cells off (half_ok = 0)
    const int ct = unit_cell_type<REV>(P, pos0, npairs);
    if (!NM && !TR && ct == kCellF16) {
        if constexpr (!NM && !TR) {
            for (int ps = 0; ps < passes; ++ps)
                run_unit<K, kCellF16, REV, false, BAND, false>(P, qs, ts, qm, tm, pos0, pos0 + npairs,
                                                  ps * fit, min(fit, G - ps * fit), W, slot, lds, lds_bnd);
        }
    } else if (ct == kCellU16 || ct == kCellF16) {
        for (int ps = 0; ps < passes; ++ps)
            run_unit<K, kCellU16, REV, NM, BAND, TR>(P, qs, ts, qm, tm, pos0, pos0 + npairs,
                                                     ps * fit, min(fit, G - ps * fit), W, slot,
                                                     lds, lds_bnd);
    } else {
        for (int it = 0; it < 2 * passes; ++it) {
            const int half = it / passes, ps = it % passes;
            run_unit<K, kCellWide, REV, NM, BAND, TR>(P, qs, ts, qm, tm, pos0 + (int64_t)half * G,
                                            pos0 + npairs, ps * fit, min(fit, G - ps * fit), W,
                                            slot, lds, lds_bnd);
        }
    }
}

// Resident waves per SIMD each width is compiled for: 512 VGPRs per lane
// hold three waves of at most 168 registers (K <= 16, N masks included) or
// two of at most 256 (K = 32).  The trace pass keeps three only at K = 8
// (its choice codes take registers of their own).  The host sizes the grid
// to match.
template <int K, bool NM = false, bool TR = false>
constexpr int kMinWaves = TR ? (K <= 8 ? 3 : 2) : (K <= 16 ? 3 : 2);

// Plain mode: pairs in input order, fixed lanes/cols, units of 128/W pairs
// dealt to waves round robin.
template <int K, bool NM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMinWaves<K, NM>, 8))) void plain_kernel(KParams P, int W) {
    __shared__ __attribute__((aligned(16))) uint32_t lds_saved[kWave * 2 * K];
    __shared__ __attribute__((aligned(16))) uint32_t lds_bnd[kBndLdsBytes / 4];
    BaseStream qs, ts, qm, tm;
    qs.init(P.q_seqs, P.q_off, P.n_pairs);
    ts.init(P.t_seqs, P.t_off, P.n_pairs);
    qm.init_mask(P.q_nmask, P.q_off, P.n_pairs);
    tm.init_mask(P.t_nmask, P.t_off, P.n_pairs);
    const int ppu = 2 * (kWave / W);
    const int64_t n_units = (P.n_pairs + ppu - 1) / ppu;
    uint32_t *slot = P.scratch + (size_t)blockIdx.x * (size_t)P.slot_words;
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int64_t pos0 = u * ppu;
        const int np = (int)min<int64_t>(ppu, P.n_pairs - pos0);
        process_unit<K, false, NM, false, false>(P, qs, ts, qm, tm, pos0, np, W, slot, lds_saved,
                                                 lds_bnd);
    }
}

// Sleeps of 127 * 64 clocks (about 3.4 us) per wave slot before a
// persistent wave's first claim.
constexpr int kClaimStagger = 4;

// Persistent mode: one launch; each wave claims units (a run of
// near-equal pairs of one length bin, in descending cost order) from an
// atomic counter until the planned units are exhausted.  The lane-group
// width comes from the unit's bin; the query columns per lane (K) are fixed
// per launch so every width shares one register budget.  REV is the start
// pass (reversed prefixes ending at the forward answers); NM reads N masks;
// BAND restricts the table to a diagonal band; TR is the trace pass.
template <int K, bool REV, bool NM, bool BAND, bool TR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMinWaves<K, NM, TR>, 8))) void persistent_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) uint32_t lds_saved[kWave * 2 * K];
    __shared__ __attribute__((aligned(16))) uint32_t lds_bnd[kBndLdsBytes / 4];
    BaseStream qs, ts, qm, tm;
    qs.init(P.q_seqs, P.q_off, P.n_pairs);
    ts.init(P.t_seqs, P.t_off, P.n_pairs);
    qm.init_mask(P.q_nmask, P.q_off, P.n_pairs);
    tm.init_mask(P.t_nmask, P.t_off, P.n_pairs);
    uint32_t *slot = P.scratch + (size_t)blockIdx.x * (size_t)P.slot_words;
    const int lane = threadIdx.x & (kWave - 1);
    // this launch claims the units of the bins with K query columns per lane
    constexpr int kc = K == 8 ? 0 : K == 16 ? 1 : 2;
    int32_t *const counter = P.unit_counter + kc;
    const int total = __builtin_amdgcn_readfirstlane(P.total_units[kc]);
    // Spread the first claims over the SIMDs.  The queue starts with the
    // costliest units; left to arrival order, the waves dispatched first
    // (several to a SIMD) take them, and a batch with fewer long units than
    // SIMDs runs them stacked.  A wave that is not in its SIMD's first wave
    // slot (HW_ID.WAVE_ID > 0) sleeps a few microseconds per slot before
    // its first claim, and stops sleeping once every unit is claimed (a
    // small batch then ends as soon as its work does).  Timed sleeps: no
    // wave waits on another.
    {
        const int slot_id = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 4) & 15;
        const int naps = min(slot_id, 3) * kClaimStagger;
        for (int k = 0; k < naps; ++k) {
            __builtin_amdgcn_s_sleep(127);
            const int claimed = __builtin_amdgcn_readfirstlane(
                __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (claimed >= total) break;
        }
    }
    for (;;) {
        int u = 0;
        if (lane == 0) u = atomicAdd(counter, 1);
        u = __builtin_amdgcn_readfirstlane(__shfl(u, 0, kWave));
        if (u >= total) break;
        int b = 0;
        for (int k = 0; k < kMaxBins; ++k) {
            const int u0 = P.bins[k].unit0, nu = P.bins[k].units;
            if (!P.bins[k].split && P.bins[k].cols == K && u >= u0 && u < u0 + nu) b = k;
        }
        b = __builtin_amdgcn_readfirstlane(b);
        const BinDesc &bd = P.bins[b];
        const int lanes = __builtin_amdgcn_readfirstlane(bd.lanes);
        const int ppu = __builtin_amdgcn_readfirstlane(bd.pairs);
        const int64_t first = __builtin_amdgcn_readfirstlane(bd.first);
        const int64_t count = __builtin_amdgcn_readfirstlane(bd.count);
        const int64_t pos0 = first + (int64_t)(u - __builtin_amdgcn_readfirstlane(bd.unit0)) * ppu;
        const int np = (int)min<int64_t>(ppu, first + count - pos0);
        process_unit<K, REV, NM, BAND, TR>(P, qs, ts, qm, tm, pos0, np, lanes, slot, lds_saved,
                                           lds_bnd);
    }
}

// A strip needs at least this many rows to be worth a wave of its own.
constexpr int kMinStripRows = 256;

// The split class (calls with split_waves set): units of 64-lane bins, each
// run by NW waves of one workgroup, one strip of target rows per wave (the
// protocol is at SplitCtx).  A workgroup claims units from the class's
// counter; a unit with too few rows, or with 32-bit cells, runs on the
// workgroup's first wave alone.  The strips' bests merge into the first
// maximum over the whole table (the strips are row ranges in order, and
// the 64-bit keys order by score, then first row, then first column).
// (two resident waves per SIMD: the kernel holds the split and the
// single-wave unit code, and needs more than three waves' share of
// registers without spilling)
template <int K, int NW>
__global__ __launch_bounds__(kWave * NW) __attribute__((amdgpu_waves_per_eu(2, 8))) void split_kernel(KParams P) {
    __shared__ __attribute__((aligned(16))) uint32_t lds_saved[NW][kWave * 2 * K];
    __shared__ __attribute__((aligned(16))) uint32_t lds_bnd[NW][kBndLdsBytes / 4];
    __shared__ int32_t s_prod[NW], s_cons[NW];
    __shared__ int32_t s_fail, s_unit;
    __shared__ unsigned long long s_keys[2 * NW];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    BaseStream qs, ts, qm, tm;
    qs.init(P.q_seqs, P.q_off, P.n_pairs);
    ts.init(P.t_seqs, P.t_off, P.n_pairs);
    qm.init_mask(nullptr, P.q_off, P.n_pairs);
    tm.init_mask(nullptr, P.t_off, P.n_pairs);
    const size_t sw = (size_t)P.slot_words;
    uint32_t *slot = P.scratch + ((size_t)blockIdx.x * NW + wv) * sw;
    int32_t *const counter = P.unit_counter + kSplitClass;
    const int total = __builtin_amdgcn_readfirstlane(P.total_units[kSplitClass]);
    for (;;) {
        if (threadIdx.x == 0) {
            s_unit = atomicAdd(counter, 1);
            s_fail = 0;
        }
        if (threadIdx.x < NW) {
            s_prod[threadIdx.x] = 0;
            s_cons[threadIdx.x] = 0;
        }
        if (threadIdx.x < 2 * NW) s_keys[threadIdx.x] = 0ull;
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(s_unit);
        if (u >= total) break;
        int b = 0;
        for (int k = 0; k < kMaxBins; ++k) {
            const int u0 = P.bins[k].unit0, nu = P.bins[k].units;
            if (P.bins[k].split && u >= u0 && u < u0 + nu) b = k;
        }
        b = __builtin_amdgcn_readfirstlane(b);
        const BinDesc &bd = P.bins[b];
        const int lanes = __builtin_amdgcn_readfirstlane(bd.lanes);
        const int ppu = __builtin_amdgcn_readfirstlane(bd.pairs);
        const int64_t first = __builtin_amdgcn_readfirstlane(bd.first);
        const int64_t count = __builtin_amdgcn_readfirstlane(bd.count);
        const int64_t pos0 =
            first + (int64_t)(u - __builtin_amdgcn_readfirstlane(bd.unit0)) * ppu;
        const int np = (int)min<int64_t>(ppu, first + count - pos0);
        // the unit's rows and cell type (the same in every wave)
        int rmax = 0;
        for (int k = lane; k < np; k += kWave)
            rmax = max(rmax, load_pair<false>(P, pos0 + k, pos0 + np, true).n);
        const int R = wave_max(rmax);
        const int ct = unit_cell_type<false>(P, pos0, np);
        const int nw = (ct == kCellWide || lanes != kWave) ? 1
                                                           : min(NW, max(1, R / kMinStripRows));
        if (nw == 1) {
            if (wv == 0)
                process_unit<K, false, false, false, false>(P, qs, ts, qm, tm, pos0, np, lanes,
                                                            slot, lds_saved[0], lds_bnd[0]);
        } else if (wv < nw) {
            const int rs = (R + nw - 1) / nw;
            SplitCtx sp;
            sp.nw = nw;
            sp.ws = wv;
            sp.r_lo = wv * rs;
            sp.r_hi = min(R, (wv + 1) * rs);
            sp.ring = slot + sw / 2;
            sp.ring_above =
                wv > 0 ? P.scratch + ((size_t)blockIdx.x * NW + wv - 1) * sw + sw / 2 : nullptr;
            sp.prod = s_prod;
            sp.cons = s_cons;
            sp.fail = &s_fail;
            sp.keys = s_keys;
            if (ct == kCellF16)
                run_unit<K, kCellF16, false, false, false, false, true>(
                    P, qs, ts, qm, tm, pos0, pos0 + np, 0, 1, kWave, slot, lds_saved[wv],
                    lds_bnd[wv], &sp);
            else
                run_unit<K, kCellU16, false, false, false, false, true>(
                    P, qs, ts, qm, tm, pos0, pos0 + np, 0, 1, kWave, slot, lds_saved[wv],
                    lds_bnd[wv], &sp);
        }
        __syncthreads();
        if (nw > 1 && wv == 0 && lane < 2) {
            unsigned long long key = 0ull;
            for (int w = 0; w < nw; ++w) key = max(key, s_keys[w * 2 + lane]);
            PairRef pr = load_pair<false>(P, pos0 + lane, pos0 + np, true);
            if (s_fail) pr.invalid = true;
            write_result<false>(P, pr, key);
            signal_done(P, pr.id);
        }
        __syncthreads();
    }
}

}  // namespace

bool plain_variant_exists(int lanes, int cols) {
    const bool w = lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16 ||
                   lanes == 32 || lanes == 64;
    return w && (cols == 8 || cols == 16 || cols == 32);
}

template <bool NM>
hipError_t launch_plain_nm(const KParams &p, int lanes, int cols, int grid, hipStream_t stream) {
    if (cols == 32)
        hipLaunchKernelGGL((plain_kernel<32, NM>), dim3(grid), dim3(kWave), 0, stream, p, lanes);
    else if (cols == 16)
        hipLaunchKernelGGL((plain_kernel<16, NM>), dim3(grid), dim3(kWave), 0, stream, p, lanes);
    else if (cols == 8)
        hipLaunchKernelGGL((plain_kernel<8, NM>), dim3(grid), dim3(kWave), 0, stream, p, lanes);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_plain(const KParams &p, int lanes, int cols, int grid, hipStream_t stream) {
    if (p.q_nmask || p.t_nmask) return launch_plain_nm<true>(p, lanes, cols, grid, stream);
    return launch_plain_nm<false>(p, lanes, cols, grid, stream);
}

bool persistent_lanes_supported(int lanes) {
    return lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 ||
           lanes == 64;
}

template <bool REV, bool NM, bool BAND = false, bool TR = false>
hipError_t launch_persistent_t(const KParams &p, int cols, int grid, hipStream_t stream) {
    // the trace pass has no 32-column kernel (its codes would spill)
    if (cols == 32) {
        if constexpr (!TR)
            hipLaunchKernelGGL((persistent_kernel<32, REV, NM, BAND, TR>), dim3(grid),
                               dim3(kWave), 0, stream, p);
        else
            return hipErrorInvalidValue;
    } else if (cols == 16)
        hipLaunchKernelGGL((persistent_kernel<16, REV, NM, BAND, TR>), dim3(grid), dim3(kWave),
                           0, stream, p);
    else if (cols == 8)
        hipLaunchKernelGGL((persistent_kernel<8, REV, NM, BAND, TR>), dim3(grid), dim3(kWave),
                           0, stream, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_split(const KParams &p, int cols, int waves, int grid, hipStream_t stream) {
    if (cols != 16 || waves != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL((split_kernel<16, 4>), dim3(grid), dim3(kWave * 4), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_persistent(const KParams &p, int cols, int grid, hipStream_t stream) {
    const bool nm = p.q_nmask || p.t_nmask;
    if (p.band >= 0) {
        if (nm || p.in_score) return hipErrorInvalidValue;
        return launch_persistent_t<false, false, true>(p, cols, grid, stream);
    }
    if (p.cig != nullptr) {
        if (nm || !p.in_score || !p.in_qstart || cols == 32) return hipErrorInvalidValue;
        return launch_persistent_t<false, false, false, true>(p, cols, grid, stream);
    }
    if (p.in_score)
        return nm ? launch_persistent_t<true, true>(p, cols, grid, stream)
                  : launch_persistent_t<true, false>(p, cols, grid, stream);
    return nm ? launch_persistent_t<false, true>(p, cols, grid, stream)
              : launch_persistent_t<false, false>(p, cols, grid, stream);
}

}  // namespace salo
