/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Reference for the GPU packing step.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call it; the
 * product path never links it.
 *
 * What it computes: reads arrive as one character per base (SALoBa,
 * Section II-B: eight bits per base in read data), and every method of the
 * evaluation packs them on the device before extension (Section V-A).  This
 * build's packed format is 2 bits per base: A=0 C=1 G=2 T=3, base k of the
 * output stream in byte k>>2 at bits 2*(k&3) (least significant pair
 * first), the same convention the aligner reads.
 *
 *   - chars[0 .. n_chars) holds the concatenated sequences; sequence s is
 *     chars[off[s] .. off[s+1]), with off non-decreasing, off[0] = 0 and
 *     off[n_seqs] = n_chars (revcomp only; forward packing ignores off).
 *   - Output base k is the code of chars[k] (forward), or, with revcomp,
 *     the complement (3 - code) of the character mirrored inside its
 *     sequence: chars[off[s] + off[s+1] - 1 - k] for off[s] <= k < off[s+1].
 *   - A, C, G, T are accepted in either case.  Any other character is
 *     counted as invalid and its base is written as 0 (A), with or without
 *     revcomp.  With revcomp, a base k that no sequence covers (offsets
 *     that break the rule above) is also written as 0 and counted.
 *   - The output is ceil(n_chars / 16) 32-bit words; bits past the last
 *     base are 0.
 *
 * Plain byte-at-a-time code: every step is the definition above.
 */
#include <stdint.h>
#include <string.h>

static int char_code(uint8_t c, int *code) {
    switch (c) {
    case 'A': case 'a': *code = 0; return 1;
    case 'C': case 'c': *code = 1; return 1;
    case 'G': case 'g': *code = 2; return 1;
    case 'T': case 't': *code = 3; return 1;
    default: *code = 0; return 0;
    }
}

/* Returns the number of invalid bases; writes ceil(n_chars/16)*4 bytes.
 * With nmask (ceil(n_chars/32) 32-bit words, or NULL): N and n are bases,
 * written as 0 with bit k of the mask set (the complement of N is N);
 * without it they are invalid like any other character. */
int64_t oracle_pack_n(const uint8_t *chars, int64_t n_chars, const int64_t *off,
                      int64_t n_seqs, int revcomp, uint8_t *out, uint32_t *nmask) {
    const int64_t out_bytes = ((n_chars + 15) / 16) * 4;
    memset(out, 0, (size_t)out_bytes);
    if (nmask) memset(nmask, 0, (size_t)((n_chars + 31) / 32) * 4);
    int64_t invalid = 0;
    int64_t s = 0;                     /* sequence holding base k (revcomp) */
    for (int64_t k = 0; k < n_chars; ++k) {
        int code = 0, ok = 0;
        int64_t src = k;
        if (!revcomp) {
            ok = char_code(chars[k], &code);
        } else {
            src = -1;
            while (s < n_seqs && off[s + 1] <= k) ++s;
            if (s < n_seqs && off[s] <= k && k < off[s + 1]) {
                src = off[s] + off[s + 1] - 1 - k;
                ok = char_code(chars[src], &code);
                if (ok) code = 3 - code;
            }
        }
        if (!ok && nmask && src >= 0 && (chars[src] == 'N' || chars[src] == 'n')) {
            nmask[k >> 5] |= 1u << (k & 31);
            ok = 1;
            code = 0;
        }
        if (!ok) {
            ++invalid;
            code = 0;
        }
        out[k >> 2] |= (uint8_t)(code << (2 * (k & 3)));
    }
    return invalid;
}

/* Without an N mask. */
int64_t oracle_pack(const uint8_t *chars, int64_t n_chars, const int64_t *off,
                    int64_t n_seqs, int revcomp, uint8_t *out) {
    return oracle_pack_n(chars, n_chars, off, n_seqs, revcomp, out, NULL);
}
