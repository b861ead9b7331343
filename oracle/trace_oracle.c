/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Reference for the GPU trace pass.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call it; the
 * product path never links it.
 *
 * What it computes: the answer of Eq. 1 (SALoBa, Section II-A) is the
 * highest cell and the path that reaches it (the trace of the highest
 * score).  Given a pair's score S > 0, its end (q_end, t_end) and its start
 * (q_start, t_start) from the start-position oracle, this function returns
 * one optimal alignment between them as a run-length CIGAR.
 *
 * Definition used: the textbook three-matrix Gotoh recurrence over the
 * sub-table rows t_start..t_end and columns q_start..q_end, anchored at the
 * start (the first aligned pair is (t_start, q_start)).  With 1-based local
 * indices i = 1..n', j = 1..m':
 *     E(i,j) = max{ H(i,j-1) - alpha, E(i,j-1) - beta }      (gap in the target: I)
 *     F(i,j) = max{ H(i-1,j) - alpha, F(i-1,j) - beta }      (gap in the query: D)
 *     H(i,j) = max{ H(i-1,j-1) + S(i,j), E(i,j), F(i,j) }   (no 0 floor)
 * with H(0,0) = 0 and every other boundary value minus infinity, so H(n',m')
 * is the best score of an alignment from the start to the end; it must be S.
 *
 * The trace walks back from (n', m') in state H and at every step takes the
 * first option, in this order, that reproduces the cell's value:
 *     state H: the aligned pair (diagonal), then E (an I ends here), then F (a D ends here);
 *     state E: the gap opens here (from H(i,j-1)), then it extends (from E(i,j-1));
 *     state F: the gap opens here (from H(i-1,j)), then it extends (from F(i-1,j)).
 * Taking the first value-preserving option at every step gives, among all
 * optimal paths, the one whose sequence of choices is smallest in that order.
 *
 * CIGAR: one uint32 per run, (length << 4) | op, with the BAM operation
 * codes '=' 7 (equal bases), 'X' 8 (unequal bases), 'I' 1 (query base
 * against a gap in the target), 'D' 2 (target base against a gap in the
 * query); runs in the order of the alignment, equal neighbouring operations
 * merged.  Plain int64 arithmetic; minus infinity is INT64_MIN / 4.
 */
#include <stdint.h>
#include <stdlib.h>

#define TRACE_NEG_INF (INT64_MIN / 4)
#define OP_EQ 7
#define OP_X 8
#define OP_I 1
#define OP_D 2

static inline int trace_base(const uint8_t *packed, int64_t k)
{
    return (packed[k >> 2] >> (2 * (k & 3))) & 3;
}

static inline int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/*
 * For every pair p: cig_len[p] = number of runs written at
 * cig[cig_off[p] ..], 0 when score[p] <= 0, -1 when the pair is
 * inconsistent (H(n', m') != score, bad coordinates) or the runs do not fit
 * cig_off[p+1] - cig_off[p].  Returns the number of such pairs, or -1 when
 * memory runs out.
 */
int64_t oracle_trace_batch(const uint8_t *q_seqs, const int64_t *q_off,
                           const uint8_t *t_seqs, const int64_t *t_off, int64_t n_pairs,
                           int64_t match, int64_t mismatch, int64_t gap_open,
                           int64_t gap_extend, const int64_t *score, const int64_t *q_start,
                           const int64_t *q_end, const int64_t *t_start, const int64_t *t_end,
                           const int64_t *cig_off, uint32_t *cig, int64_t *cig_len)
{
    const int64_t alpha = gap_open + gap_extend, beta = gap_extend;
    int64_t bad = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        cig_len[p] = 0;
        if (score[p] <= 0) continue;
        const int64_t m = q_off[p + 1] - q_off[p], n = t_off[p + 1] - t_off[p];
        const int64_t qs = q_start[p], qe = q_end[p], ts = t_start[p], te = t_end[p];
        if (qs < 0 || qs > qe || qe >= m || ts < 0 || ts > te || te >= n) {
            cig_len[p] = -1;
            ++bad;
            continue;
        }
        const int64_t mm = qe - qs + 1, nn = te - ts + 1, w = mm + 1;
        const size_t cells = (size_t)(nn + 1) * (size_t)w;
        int64_t *H = (int64_t *)malloc(sizeof(int64_t) * cells);
        int64_t *E = (int64_t *)malloc(sizeof(int64_t) * cells);
        int64_t *F = (int64_t *)malloc(sizeof(int64_t) * cells);
        uint32_t *rev = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(mm + nn));
        if (!H || !E || !F || !rev) {
            free(H); free(E); free(F); free(rev);
            return -1;
        }
#define AT(A, i, j) A[(size_t)(i) * (size_t)w + (size_t)(j)]
        for (int64_t i = 0; i <= nn; ++i)
            for (int64_t j = 0; j <= mm; ++j) {
                AT(H, i, j) = TRACE_NEG_INF;
                AT(E, i, j) = TRACE_NEG_INF;
                AT(F, i, j) = TRACE_NEG_INF;
            }
        AT(H, 0, 0) = 0;
        for (int64_t i = 1; i <= nn; ++i) {
            const int ti = trace_base(t_seqs, t_off[p] + ts + i - 1);
            for (int64_t j = 1; j <= mm; ++j) {
                const int qj = trace_base(q_seqs, q_off[p] + qs + j - 1);
                const int64_t s = ti == qj ? match : mismatch;
                AT(E, i, j) = max2(max2(AT(H, i, j - 1) - alpha, AT(E, i, j - 1) - beta),
                                   TRACE_NEG_INF);
                AT(F, i, j) = max2(max2(AT(H, i - 1, j) - alpha, AT(F, i - 1, j) - beta),
                                   TRACE_NEG_INF);
                AT(H, i, j) = max2(max2(AT(H, i - 1, j - 1) + s, AT(E, i, j)), AT(F, i, j));
            }
        }
        int ok = AT(H, nn, mm) == score[p];
        /* walk back; runs collected last-first */
        int64_t i = nn, j = mm, nrev = 0, run_len = 0;
        int run_op = -1, state = 0;          /* 0: H, 1: E, 2: F */
        while (ok && (i > 0 || j > 0)) {
            int op;
            /* every value on row 0 or column 0 but the anchor is minus
             * infinity: a walk that reaches one has lost the path */
            if (i <= 0 || j <= 0) { ok = 0; break; }
            if (state == 0) {
                const int ti = trace_base(t_seqs, t_off[p] + ts + i - 1);
                const int qj = trace_base(q_seqs, q_off[p] + qs + j - 1);
                const int64_t s = ti == qj ? match : mismatch;
                if (AT(H, i, j) == AT(H, i - 1, j - 1) + s) {
                    op = ti == qj ? OP_EQ : OP_X;
                    --i;
                    --j;
                } else if (AT(H, i, j) == AT(E, i, j)) {
                    state = 1;
                    continue;
                } else {
                    state = 2;
                    continue;
                }
            } else if (state == 1) {
                op = OP_I;
                if (AT(E, i, j) == AT(H, i, j - 1) - alpha) state = 0;
                --j;
            } else {
                op = OP_D;
                if (AT(F, i, j) == AT(H, i - 1, j) - alpha) state = 0;
                --i;
            }
            if (op == run_op) {
                ++run_len;
            } else {
                if (run_op >= 0) rev[nrev++] = (uint32_t)(run_len << 4) | (uint32_t)run_op;
                run_op = op;
                run_len = 1;
            }
        }
        /* the walk must end at the anchor in state H */
        if (ok && state != 0) ok = 0;
        if (ok && run_op >= 0) rev[nrev++] = (uint32_t)(run_len << 4) | (uint32_t)run_op;
        if (ok && nrev > cig_off[p + 1] - cig_off[p]) ok = 0;
        if (ok) {
            for (int64_t k = 0; k < nrev; ++k) cig[cig_off[p] + k] = rev[nrev - 1 - k];
            cig_len[p] = nrev;
        } else {
            cig_len[p] = -1;
            ++bad;
        }
#undef AT
        free(H); free(E); free(F); free(rev);
    }
    return bad;
}
