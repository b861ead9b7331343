/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Reference for the GPU banded pass.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may build, load or call it; the
 * product path never links it.
 *
 * What it computes (SALoBa, Section VII-B: banded seed extension fills only
 * the cells within a fixed width of the diagonal): Eq. 1 restricted to the
 * band |i - j| <= w, i over target bases, j over query bases.  A cell
 * outside the band does not exist: as a neighbour it behaves like the
 * table's boundary (H = 0, E = F = minus infinity), and it is never a
 * candidate for the answer.  Inside the band every cell follows Eq. 1
 * exactly as in the unbanded oracle (alpha = gap_open + gap_extend,
 * beta = gap_extend, the 0 floor, the first maximum in row-major order,
 * (-1, -1) for a score of 0).  A band at least max(m, n) wide gives the
 * unbanded answer.
 *
 * Plain full-table loops with an in-band test per cell; int64 arithmetic.
 */
#include <stdint.h>
#include <stdlib.h>

#define BAND_NEG_INF (INT64_MIN / 4)

static inline int band_base(const uint8_t *packed, int64_t k)
{
    return (packed[k >> 2] >> (2 * (k & 3))) & 3;
}

static inline int in_band(int64_t i, int64_t j, int64_t w)
{
    const int64_t d = i - j;
    return d <= w && d >= -w;
}

/* Returns 0, or -1 when memory runs out.  w < 0 is not allowed (the caller
 * checks). */
int oracle_align_banded(const uint8_t *q_seqs, const int64_t *q_off,
                        const uint8_t *t_seqs, const int64_t *t_off,
                        int64_t n_pairs, int64_t match, int64_t mismatch,
                        int64_t gap_open, int64_t gap_extend, int64_t w,
                        int64_t *out_score, int64_t *out_qend, int64_t *out_tend)
{
    const int64_t alpha = gap_open + gap_extend, beta = gap_extend;
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int64_t q0 = q_off[p], m = q_off[p + 1] - q0;
        const int64_t t0 = t_off[p], n = t_off[p + 1] - t0;
        int64_t best = 0, bi = -1, bj = -1;
        if (m > 0 && n > 0) {
            int64_t *Hrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
            int64_t *Frow = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
            if (!Hrow || !Frow) { free(Hrow); free(Frow); return -1; }
            for (int64_t j = 0; j < m; ++j) { Hrow[j] = 0; Frow[j] = BAND_NEG_INF; }
            for (int64_t i = 0; i < n; ++i) {
                const int ti = band_base(t_seqs, t0 + i);
                int64_t h_left = 0, e = BAND_NEG_INF, h_diag = 0;
                for (int64_t j = 0; j < m; ++j) {
                    int64_t h, f;
                    if (!in_band(i, j, w)) {
                        /* not a cell: boundary values for its neighbours */
                        h = 0;
                        f = BAND_NEG_INF;
                        e = BAND_NEG_INF;
                    } else {
                        const int qj = band_base(q_seqs, q0 + j);
                        const int64_t s = (ti == qj) ? match : mismatch;
                        const int64_t e_open = h_left - alpha, e_ext = e - beta;
                        e = e_open > e_ext ? e_open : e_ext;
                        const int64_t f_open = Hrow[j] - alpha, f_ext = Frow[j] - beta;
                        f = f_open > f_ext ? f_open : f_ext;
                        h = h_diag + s;
                        if (e > h) h = e;
                        if (f > h) h = f;
                        if (h < 0) h = 0;
                        if (h > best) { best = h; bi = i; bj = j; }
                    }
                    h_diag = Hrow[j];
                    Hrow[j] = h;
                    Frow[j] = f;
                    h_left = h;
                }
            }
            free(Hrow);
            free(Frow);
        }
        out_score[p] = best;
        out_qend[p] = best > 0 ? bj : -1;
        out_tend[p] = best > 0 ? bi : -1;
    }
    return 0;
}
