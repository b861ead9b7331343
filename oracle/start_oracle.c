/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Reference for the GPU start-position pass.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may build, load or call
 * it; the product path never links it.
 *
 * What it computes: the answer of Eq. 1 (SALoBa, Section II-A) is the
 * highest cell and the path that reaches it ("the trace of the highest
 * score").  The end of that path is (q_end, t_end) from the alignment
 * oracle; this function finds where the path begins.
 *
 * Reading (the paper does not spell it out): for a pair whose best score S
 * > 0 ends at (q_end, t_end), run the Gotoh recurrence backwards from that
 * cell, anchored there.  Over the reversed prefixes
 *     rq[j'] = q[q_end - j'],  rt[i'] = t[t_end - i']   (0 <= j' <= q_end, 0 <= i' <= t_end)
 * it computes
 *     A(i',j') = max{ E(i',j'), F(i',j'), A(i'-1,j'-1) + S(i',j') }   (no 0 floor)
 *     E(i',j') = max{ A(i',j'-1) - alpha, E(i',j'-1) - beta }
 *     F(i',j') = max{ A(i'-1,j') - alpha, F(i'-1,j') - beta }
 * with A(-1,-1) = 0 and every other boundary value minus infinity.
 * A(i',j') is the best score of an alignment whose last aligned pair is
 * (q_end, t_end) and whose first is (q_end - j', t_end - i'), so the
 * table's maximum is S.  The answer is the first cell reaching S in
 * row-major order over (i', j'): among the optimal alignments ending at
 * (q_end, t_end), the start with the largest t_start, then the largest
 * q_start.  Outputs q_start = q_end - j', t_start = t_end - i'; pairs with
 * S = 0 get (-1, -1).
 *
 * Because (q_end, t_end) is the first maximum of the whole table, every
 * alignment scoring S inside the prefix rectangle ends at that cell, so the
 * anchor (and the absence of the 0 floor) never changes the answer: the
 * local recurrence over the reversed prefixes gives the same start.  The
 * tests check both formulations against each other.
 *
 * alpha = gap_open + gap_extend and beta = gap_extend, as in the alignment
 * oracle.  Plain int64 arithmetic; minus infinity is INT64_MIN / 4.
 */
#include <stdint.h>
#include <stdlib.h>

#define START_NEG_INF (INT64_MIN / 4)

static inline int start_base(const uint8_t *packed, int64_t k)
{
    return (packed[k >> 2] >> (2 * (k & 3))) & 3;
}

/* Optional N masks (bit k of word k>>5): an N scores mismatch against
 * every base, N included. */
static inline int start_is_n(const uint32_t *mask, int64_t k)
{
    return mask != NULL && ((mask[k >> 5] >> (k & 31)) & 1u);
}

/*
 * For every pair p with score[p] > 0, writes q_start / t_start (else -1).
 * Returns the number of pairs whose anchored maximum differed from score[p]
 * (0 when the inputs are the alignment oracle's answers), or -1 when memory
 * runs out.
 */
int64_t oracle_start_batch_n(const uint8_t *q_seqs, const uint32_t *q_nmask,
                             const int64_t *q_off,
                             const uint8_t *t_seqs, const uint32_t *t_nmask,
                             const int64_t *t_off,
                             int64_t n_pairs, int64_t match, int64_t mismatch,
                             int64_t gap_open, int64_t gap_extend,
                             const int64_t *score, const int64_t *qend, const int64_t *tend,
                             int64_t *out_qstart, int64_t *out_tstart)
{
    const int64_t alpha = gap_open + gap_extend, beta = gap_extend;
    int64_t bad = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        out_qstart[p] = -1;
        out_tstart[p] = -1;
        if (score[p] <= 0) continue;
        const int64_t qe = qend[p], te = tend[p];
        const int64_t mq = qe + 1;                 /* reversed query length */
        int64_t *Arow = (int64_t *)malloc(sizeof(int64_t) * (size_t)mq);
        int64_t *Frow = (int64_t *)malloc(sizeof(int64_t) * (size_t)mq);
        if (!Arow || !Frow) { free(Arow); free(Frow); return -1; }
        for (int64_t j = 0; j < mq; ++j) {
            Arow[j] = START_NEG_INF;               /* A(-1, j') */
            Frow[j] = START_NEG_INF;               /* F(-1, j') */
        }
        int64_t best = START_NEG_INF, bi = -1, bj = -1;
        for (int64_t i = 0; i <= te; ++i) {
            const int ti = start_base(t_seqs, t_off[p] + te - i);
            const int t_is_n = start_is_n(t_nmask, t_off[p] + te - i);
            int64_t a_left = START_NEG_INF;        /* A(i', -1) */
            int64_t e = START_NEG_INF;             /* E(i', -1) */
            int64_t a_diag = i == 0 ? 0 : START_NEG_INF;   /* A(i'-1, -1): the anchor */
            for (int64_t j = 0; j < mq; ++j) {
                const int qj = start_base(q_seqs, q_off[p] + qe - j);
                const int64_t s_acgt = (ti == qj) ? match : mismatch;
                const int64_t s =
                    (t_is_n || start_is_n(q_nmask, q_off[p] + qe - j)) ? mismatch : s_acgt;
                const int64_t e_open = a_left - alpha, e_ext = e - beta;
                e = e_open > e_ext ? e_open : e_ext;
                const int64_t f_open = Arow[j] - alpha, f_ext = Frow[j] - beta;
                const int64_t f = f_open > f_ext ? f_open : f_ext;
                int64_t a = a_diag + s;
                if (e > a) a = e;
                if (f > a) a = f;
                a_diag = Arow[j];
                Arow[j] = a;
                Frow[j] = f;
                a_left = a;
                if (a > best) { best = a; bi = i; bj = j; }
            }
        }
        free(Arow);
        free(Frow);
        if (best != score[p]) ++bad;
        out_qstart[p] = qe - bj;
        out_tstart[p] = te - bi;
    }
    return bad;
}

/* Without N masks. */
int64_t oracle_start_batch(const uint8_t *q_seqs, const int64_t *q_off,
                           const uint8_t *t_seqs, const int64_t *t_off,
                           int64_t n_pairs, int64_t match, int64_t mismatch,
                           int64_t gap_open, int64_t gap_extend,
                           const int64_t *score, const int64_t *qend, const int64_t *tend,
                           int64_t *out_qstart, int64_t *out_tstart)
{
    return oracle_start_batch_n(q_seqs, NULL, q_off, t_seqs, NULL, t_off, n_pairs, match,
                                mismatch, gap_open, gap_extend, score, qend, tend,
                                out_qstart, out_tstart);
}
