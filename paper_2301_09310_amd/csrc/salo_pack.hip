// Packing kernels: character reads (one byte per base) into the 2-bit
// stream the aligner reads (A=0 C=1 G=2 T=3, base k in byte k>>2 at bits
// 2*(k&3)), optionally reverse-complemented per sequence.
//
// Why on the device: read data stores a base per byte (SALoBa,
// Section II-B), and the evaluation packs reads on the GPU for every
// method because that step alone decided a library's lead (Section V-A).
// Packing is a streaming pass: n bytes in, n/4 bytes out, so it is bound
// by HBM bandwidth.
//
// Mapping: 256 threads per block.  Forward packing: one thread per output
// 32-bit word (16 bases), reading the word's 16 characters as four aligned
// dwords.  Reverse-complement packing needs the sequence of every output
// base.  A block packs 8 words per thread.  It finds the sequences of its
// first and last bases (a 64-lane search each), stages the offsets between
// them in LDS, and builds a table of each word's sequence there.  The
// mirrored characters of a word are contiguous (in reverse), so the reads
// stay within a few cache lines.
#include "salo_internal.h"

namespace salo {
namespace {

constexpr int kPackThreads = 256;
// reverse complement: words per thread (the block's sequence search and
// offset staging are paid once for kRcWords * kPackThreads words) and
// sequence offsets staged per block
constexpr int kRcWords = 8;
constexpr int kWin = 1024;

// 2-bit code of a character and whether it is A, C, G or T in either case
// (the code formula maps A/a->0, C/c->1, G/g->2, T/t->3).
__device__ __forceinline__ uint32_t char_code(uint32_t c, bool &ok) {
    const uint32_t l = c | 0x20u;
    ok = l == 'a' || l == 'c' || l == 'g' || l == 't';
    return ((c >> 1) ^ (c >> 2)) & 3u;
}

// Four characters (one per byte, byte 0 first) to four 2-bit bases in the
// low 8 bits (byte 0 -> bits 0-1), complemented when RC, invalid
// characters as 0; adds the number of invalid characters to `bad`.
//   code     = ((c >> 1) ^ (c >> 2)) & 3 per byte (A/a 0, C/c 1, G/g 2, T/t 3)
//   expected = "acgt"[code] per byte (one v_perm)
//   a byte is valid iff (c | 0x20) == expected (exact per-byte zero test)
// 0x80 in every byte of d that is zero (exact: no borrow between bytes)
__device__ __forceinline__ uint32_t zero_bytes(uint32_t d) {
    return ((((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u) ^ 0x80808080u;
}

// With NM, N and n are bases too: their code is 0 and bit b of `nbits`
// (byte b) is set; without NM they are invalid like any other character.
template <bool RC, bool NM = false>
__device__ __forceinline__ uint32_t pack4(uint32_t x, uint32_t &bad, uint32_t *nbits = nullptr) {
    const uint32_t code = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    const uint32_t expect = __builtin_amdgcn_perm(0u, 0x74676361u, code);
    const uint32_t lo = x | 0x20202020u;
    const uint32_t ok = zero_bytes(lo ^ expect);           // 0x80 in A/C/G/T bytes
    if constexpr (NM) {
        const uint32_t isn = zero_bytes(lo ^ 0x6E6E6E6Eu); // 0x80 in N/n bytes
        *nbits = ((isn >> 7) & 1u) | ((isn >> 14) & 2u) | ((isn >> 21) & 4u) |
                 ((isn >> 28) & 8u);
        bad += 4u - (uint32_t)__builtin_popcount(ok | isn);
    } else {
        bad += 4u - (uint32_t)__builtin_popcount(ok);
    }
    uint32_t c = RC ? (code ^ 0x03030303u) : code;
    c &= (ok >> 6) | (ok >> 7);                            // 0x03 in valid bytes
    return (c | (c >> 6) | (c >> 12) | (c >> 18)) & 0xFFu;
}

__device__ __forceinline__ void add_invalid(unsigned long long *invalid, uint32_t bad) {
    // one atomic per wave
    uint32_t v = bad;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v != 0u && invalid != nullptr)
        atomicAdd(invalid, (unsigned long long)v);
}

// N bits of 16 bases per thread: the even thread of each pair writes the
// 32-bit mask word (its bits low, its neighbour's high).  Every thread of
// the wave takes part in the exchange.
__device__ __forceinline__ void store_nmask(uint32_t *n_mask, int64_t w, int64_t nw,
                                            uint32_t nb16) {
    const uint32_t hi = (uint32_t)__shfl_down((int)nb16, 1, 64);
    if (w < nw && (w & 1) == 0) n_mask[w >> 1] = nb16 | (w + 1 < nw ? (hi << 16) : 0u);
}

__device__ __forceinline__ bool is_n_char(uint32_t c) { return (c | 0x20u) == 'n'; }

template <bool V4, bool NM>
__global__ __launch_bounds__(kPackThreads) void pack_forward(const uint8_t *chars, int64_t n,
                                                             uint32_t *out, uint32_t *n_mask,
                                                             unsigned long long *invalid) {
    const int64_t w = (int64_t)blockIdx.x * kPackThreads + threadIdx.x;
    const int64_t nw = (n + 15) >> 4;
    uint32_t bad = 0;
    uint32_t nb16 = 0;
    if (w < nw) {
        const int64_t p0 = w << 4;
        uint32_t word = 0;
        if (p0 + 16 <= n) {
            uint32_t x[4];
            if constexpr (V4) {      // chars 16-byte aligned: one 16-byte load
                const uint4 v = *reinterpret_cast<const uint4 *>(chars + p0);
                x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
            } else {
                const uint32_t *src = reinterpret_cast<const uint32_t *>(chars + p0);
#pragma unroll
                for (int d = 0; d < 4; ++d) x[d] = src[d];
            }
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                uint32_t nb4 = 0;
                word |= pack4<false, NM>(x[d], bad, &nb4) << (8 * d);
                nb16 |= nb4 << (4 * d);
            }
        } else {
            for (int k = 0; k < 16 && p0 + k < n; ++k) {
                bool ok;
                const uint32_t c = chars[p0 + k];
                const uint32_t code = char_code(c, ok);
                const bool isn = NM && is_n_char(c);
                bad += (ok || isn) ? 0u : 1u;
                word |= (ok ? code : 0u) << (2 * k);
                nb16 |= (isn ? 1u : 0u) << k;
            }
        }
        out[w] = word;
    }
    if constexpr (NM) store_nmask(n_mask, w, nw, nb16);
    add_invalid(invalid, bad);
}

// Largest s in [lo, hi) with off[s] <= p, or lo - 1 when off[lo] > p.
__device__ int64_t last_le(const int64_t *off, int64_t lo, int64_t hi, int64_t p) {
    int64_t a = lo, b = hi;   // answer in [a-1, b-1]
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        if (off[mid] <= p) a = mid + 1;
        else b = mid;
    }
    return a - 1;
}

// The 16 characters chars[start .. start+16) as four dwords (byte j of
// g[i] is chars[start + 4i + j]); positions outside [0, n) read as 0.
// Whole dwords are read, so the buffer must be readable up to the next
// multiple of 4 bytes past n.
__device__ __forceinline__ void gather16(const uint8_t *chars, int64_t n, int64_t start,
                                         uint32_t g[4]) {
    const int64_t a = start >> 2;                          // floor, also for negatives
    const uint32_t sh = (uint32_t)(start - (a << 2)) * 8u;
    const int64_t nwords = (n + 3) >> 2;
    const uint32_t *w32 = reinterpret_cast<const uint32_t *>(chars);
    uint32_t x[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int64_t idx = a + i;
        x[i] = (idx >= 0 && idx < nwords) ? w32[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = __builtin_amdgcn_alignbit(x[i + 1], x[i], sh);
}

// Largest s in [0, n) with off[s] <= p (off non-decreasing), or -1.  The
// 64 lanes of the calling wave probe 64 evenly spaced entries per round,
// so the range shrinks 64-fold per dependent load (4 rounds for 2M
// sequences, against 21 for a one-lane binary search).  Every lane of the
// wave calls it and gets the answer.
__device__ int64_t wave_last_le(const int64_t *off, int64_t n, int64_t p) {
    const int lane = threadIdx.x & 63;
    int64_t a = 0, b = n;   // answer = a - 1 + #{s in [a, b): off[s] <= p}
    while (b - a > 64) {
        const int64_t step = (b - a + 63) >> 6;
        const int64_t idx = a + (int64_t)lane * step;
        const bool t = idx < b && off[idx] <= p;
        const int c = __popcll(__ballot(t));
        if (c == 0) return a - 1;                 // off[a] > p; off[a-1] <= p
        const int64_t na = a + (int64_t)(c - 1) * step;
        b = min<int64_t>(b, a + (int64_t)c * step);
        a = na;
    }
    const int64_t idx = a + lane;
    const bool t = idx < b && off[idx] <= p;
    return a - 1 + __popcll(__ballot(t));
}

// Bounds [lo, hi) of sequence s: from the block's staged offsets
// (win[0 .. nwin) = off[s0 ..]) when they hold both, else from off.
__device__ __forceinline__ void seq_bounds(const int64_t *win, int64_t s0, int nwin,
                                           const int64_t *off, int64_t n_seqs, int64_t s,
                                           int64_t &lo, int64_t &hi) {
    const int64_t j = s - s0;
    if (j >= 0 && j + 1 < nwin) {
        lo = win[j];
        hi = win[j + 1];
    } else {
        lo = off[s];
        hi = off[s + 1];
    }
    (void)n_seqs;
}

template <bool NM>
__global__ __launch_bounds__(kPackThreads) void pack_revcomp(const uint8_t *chars, int64_t n,
                                                             const int64_t *off,
                                                             int64_t n_seqs, uint32_t *out,
                                                             uint32_t *n_mask,
                                                             unsigned long long *invalid) {
    __shared__ int64_t win[kWin + 1];
    __shared__ int32_t wseq[kRcWords * kPackThreads];   // window index per word
    __shared__ int32_t wave_tot[kPackThreads / 64];
    __shared__ int64_t s_first, s_last;
    constexpr int64_t kSpan = (int64_t)kRcWords * kPackThreads;   // words per block
    const int64_t w0 = (int64_t)blockIdx.x * kSpan;
    const int64_t nw = (n + 15) >> 4;
    // sequences of the block's first and last bases (off[0..n_seqs-1] are
    // starts), one wave each
    if (threadIdx.x < 64) {
        const int64_t s = n_seqs > 0 ? wave_last_le(off, n_seqs, w0 << 4) : -1;
        if (threadIdx.x == 0) s_first = s < 0 ? 0 : s;
    } else if (threadIdx.x < 128) {
        const int64_t p_end = min<int64_t>(n, (w0 + kSpan) << 4) - 1;
        const int64_t s = n_seqs > 0 ? wave_last_le(off, n_seqs, p_end) : -1;
        if (threadIdx.x == 64) s_last = s < 0 ? 0 : s;
    }
    __syncthreads();
    const int64_t s0 = s_first;
    // stage off[s0 .. s_last + 1]: the bounds of every sequence the block
    // touches (at most kWin + 1 entries; beyond them, off is read directly)
    const int nwin = (int)min<int64_t>(kWin + 1, max<int64_t>(s_last - s0 + 2, 1));
    for (int t = threadIdx.x; t < nwin; t += kPackThreads) {
        const int64_t idx = s0 + t;
        win[t] = idx <= n_seqs ? off[idx] : INT64_MAX;
    }
    for (int t = threadIdx.x; t < kSpan; t += kPackThreads) wseq[t] = -1;
    __syncthreads();
    // wseq[x] = the largest window index j with win[j] <= 16 * (w0 + x), or
    // -1: each j marks the first word whose start it covers, then an
    // inclusive max-scan carries it forward
    {
        const int64_t P0 = w0 << 4;
        for (int t = threadIdx.x; t < nwin; t += kPackThreads) {
            const int64_t v = win[t];
            if (v == INT64_MAX) continue;
            const int64_t x = v <= P0 ? 0 : ((v - P0 + 15) >> 4);
            if (x < kSpan) atomicMax(&wseq[(int)x], t);
        }
    }
    __syncthreads();
    {
        // thread t scans entries [t * kRcWords, (t + 1) * kRcWords)
        int run = -1;
        int loc[kRcWords];
#pragma unroll
        for (int k = 0; k < kRcWords; ++k) {
            run = max(run, wseq[threadIdx.x * kRcWords + k]);
            loc[k] = run;
        }
        // inclusive max-scan of the threads' totals: within the wave, then
        // across the block's waves
        int inc = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o, 64);
            if ((threadIdx.x & 63) >= o) inc = max(inc, y);
        }
        if ((threadIdx.x & 63) == 63) wave_tot[threadIdx.x >> 6] = inc;
        __syncthreads();
        int carry = __shfl_up(inc, 1, 64);
        if ((threadIdx.x & 63) == 0) carry = -1;
        for (int v = 0; v < (int)(threadIdx.x >> 6); ++v) carry = max(carry, wave_tot[v]);
#pragma unroll
        for (int k = 0; k < kRcWords; ++k)
            wseq[threadIdx.x * kRcWords + k] = max(loc[k], carry);
    }
    __syncthreads();

    uint32_t bad = 0;
    // word w0 + it * kPackThreads + threadIdx.x in round it: each round's
    // stores are contiguous, and the pairs of store_nmask stay in one wave
    for (int it = 0; it < kRcWords; ++it) {
        const int64_t w = w0 + (int64_t)it * kPackThreads + threadIdx.x;
        uint32_t nb16 = 0;
        if (w < nw) {
            const int64_t p0 = w << 4;
            uint32_t word = 0;
            // sequence of the word's first base: window index, else the table
            int64_t s;
            {
                const int j = wseq[it * kPackThreads + threadIdx.x];
                if (j >= 0 && j + 1 < nwin && p0 < win[j + 1]) s = s0 + j;
                else s = n_seqs > 0 ? last_le(off, 0, n_seqs, p0) : -1;
            }
            bool fast = false;
            if (s >= 0 && s < n_seqs && p0 + 16 <= n) {
                int64_t lo, hi;
                seq_bounds(win, s0, nwin, off, n_seqs, s, lo, hi);
                if (lo <= p0 && p0 < hi) {
                    // output base k (p = p0 + k) of sequence s comes from
                    // chars[lo + hi - 1 - p]; the word's first kb bases lie in s
                    const int64_t kb = min<int64_t>(hi - p0, 16);
                    uint32_t g[4], h[4] = {0u, 0u, 0u, 0u};
                    const int64_t A = lo + hi - 1 - p0;
                    gather16(chars, n, A - 15, g);             // g byte 15-k = chars[A - k]
                    fast = true;
                    if (kb < 16) {
                        // the rest must lie in sequence s + 1 (else three or
                        // more sequences share the word: per-base path)
                        int64_t lo2, hi2;
                        if (s + 1 < n_seqs) {
                            seq_bounds(win, s0, nwin, off, n_seqs, s + 1, lo2, hi2);
                            if (lo2 == hi && hi2 - lo2 >= 16 - kb) {
                                gather16(chars, n, lo2 + hi2 - 1 - p0 - 15, h);
                            } else {
                                fast = false;
                            }
                        } else {
                            fast = false;
                        }
                    }
                    if (fast) {
                        // merged byte j (= base 15 - j): from g for j >= 16 - kb
                        const int t = 16 - (int)kb;
    #pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int r = t - 4 * i;   // first byte of dword i taken from g
                            const uint32_t mg = r <= 0 ? 0xFFFFFFFFu
                                                       : (r >= 4 ? 0u : (0xFFFFFFFFu << (8 * r)));
                            g[i] = (g[i] & mg) | (h[i] & ~mg);
                        }
                        // base k = complement of merged byte 15 - k: bases
                        // 4q..4q+3 are dword 3-q with its bytes reversed
    #pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const uint32_t rev = __builtin_amdgcn_perm(0u, g[3 - q], 0x00010203u);
                            uint32_t nb4 = 0;
                            word |= pack4<true, NM>(rev, bad, &nb4) << (8 * q);
                            nb16 |= nb4 << (4 * q);
                        }
                    }
                }
            }
            if (!fast) {
                // per base: tails, words spanning three or more sequences, and
                // offsets that break the documented rule
                word = 0;
                nb16 = 0;
                int64_t sc = s;
                for (int k = 0; k < 16; ++k) {
                    const int64_t p = p0 + k;
                    if (p >= n) break;
                    int64_t lo = 0, hi = 0;
                    if (sc >= 0 && sc < n_seqs) seq_bounds(win, s0, nwin, off, n_seqs, sc, lo, hi);
                    while (sc >= 0 && sc + 1 < n_seqs && hi <= p) {
                        ++sc;
                        seq_bounds(win, s0, nwin, off, n_seqs, sc, lo, hi);
                    }
                    bool ok = false, isn = false;
                    uint32_t code = 0;
                    if (sc >= 0 && sc < n_seqs && lo <= p && p < hi) {
                        const int64_t src = lo + hi - 1 - p;
                        if (src >= 0 && src < n) {
                            const uint32_t c = chars[src];
                            code = 3u - char_code(c, ok);
                            isn = NM && is_n_char(c);
                        }
                    }
                    bad += (ok || isn) ? 0u : 1u;
                    word |= (ok ? code : 0u) << (2 * k);
                    nb16 |= (isn ? 1u : 0u) << k;
                }
            }
            out[w] = word;
        }
        if constexpr (NM) store_nmask(n_mask, w, nw, nb16);
    }
    add_invalid(invalid, bad);
}

}  // namespace

template <bool NM>
hipError_t launch_pack_t(const uint8_t *chars, int64_t n_chars, const int64_t *offsets,
                         int64_t n_seqs, bool revcomp, uint8_t *packed, uint32_t *n_mask,
                         unsigned long long *invalid, hipStream_t stream) {
    const int64_t nw = (n_chars + 15) >> 4;
    const int64_t blocks = (nw + kPackThreads - 1) / kPackThreads;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    uint32_t *out = reinterpret_cast<uint32_t *>(packed);
    if (revcomp)
        hipLaunchKernelGGL((pack_revcomp<NM>),
                           dim3((uint32_t)((blocks + kRcWords - 1) / kRcWords)),
                           dim3(kPackThreads), 0, stream, chars, n_chars, offsets, n_seqs, out,
                           n_mask, invalid);
    else if ((reinterpret_cast<uintptr_t>(chars) & 15) == 0)
        hipLaunchKernelGGL((pack_forward<true, NM>), dim3((uint32_t)blocks), dim3(kPackThreads),
                           0, stream, chars, n_chars, out, n_mask, invalid);
    else
        hipLaunchKernelGGL((pack_forward<false, NM>), dim3((uint32_t)blocks), dim3(kPackThreads),
                           0, stream, chars, n_chars, out, n_mask, invalid);
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t *chars, int64_t n_chars, const int64_t *offsets,
                       int64_t n_seqs, bool revcomp, uint8_t *packed, uint32_t *n_mask,
                       unsigned long long *invalid, hipStream_t stream) {
    if (n_mask)
        return launch_pack_t<true>(chars, n_chars, offsets, n_seqs, revcomp, packed, n_mask,
                                   invalid, stream);
    return launch_pack_t<false>(chars, n_chars, offsets, n_seqs, revcomp, packed, nullptr,
                                invalid, stream);
}

}  // namespace salo
