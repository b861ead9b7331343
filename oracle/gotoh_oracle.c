/*
 * CPU ORACLE -- test infrastructure only.
 *
 * This file is the correctness reference for the GPU seed-extension path.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may build, load or call it.  The product path never links it.
 *
 * What it computes (SALoBa paper, Section II-A, Eq. 1): for one
 * (query, target) pair, the affine-gap Smith-Waterman-Gotoh table
 *
 *     H(i,j) = max{ 0, E(i,j), F(i,j), H(i-1,j-1) + S(i,j) }
 *     E(i,j) = max{ H(i,j-1) - alpha, E(i,j-1) - beta }
 *     F(i,j) = max{ H(i-1,j) - alpha, F(i-1,j) - beta }
 *
 * with i indexing the reference (target) and j the query (Section II-A, the
 * sentence after Eq. 1), and the answer is the maximum H over the whole
 * table (Section II-A, the description of the example figure).
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - A gap of k bases costs gap_open + k*gap_extend, so alpha (new gap) =
 *     gap_open + gap_extend and beta (continued gap) = gap_extend.
 *   - S(i,j) = match when the bases are equal, mismatch otherwise; match > 0,
 *     mismatch <= 0 are signed scores, the gap values are magnitudes.
 *   - Boundary: H(-1,j) = H(i,-1) = 0, E(i,-1) = F(-1,j) = -infinity.
 *   - Ties: among cells with the highest H the answer is the first one in
 *     row-major order over (target row i, query column j): smallest i, then
 *     smallest j.  A score of 0 (no positive cell, or an empty sequence)
 *     returns end positions (-1, -1).
 *   - Outputs: score, q_end = j, t_end = i (0-based, inclusive).
 *
 * Arithmetic is int64 throughout; -infinity is INT64_MIN/4 so that
 * subtracting any admissible penalty cannot overflow.
 *
 * Input format (shared convention with every caller, not shared code):
 * sequences are 2-bit packed, A=0 C=1 G=2 T=3, base k of a stream stored in
 * byte k>>2 at bits 2*(k&3) (least significant pair first).  Pair p uses
 * query bases [q_off[p], q_off[p+1]) and target bases [t_off[p], t_off[p+1]).
 *
 * Batch driver: pairs are independent, so a pool of POSIX threads takes
 * pairs from a shared counter, longest first.  That is the only
 * parallelism; each pair is the plain scalar recurrence above.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NEG_INF (INT64_MIN / 4)

static inline int base_at(const uint8_t *packed, int64_t k)
{
    return (packed[k >> 2] >> (2 * (k & 3))) & 3;
}

/* N masks (optional): bit k of the 32-bit word k>>5 set means base k is N.
 * An N against any base, N included, scores mismatch. */
static inline int is_n(const uint32_t *mask, int64_t k)
{
    return mask != NULL && ((mask[k >> 5] >> (k & 31)) & 1u);
}

/* One pair, Eq. 1 row by row.  Rows i = target bases, columns j = query
 * bases.  Hrow/Frow hold row i-1 while row i is being filled. */
static void gotoh_pair(const uint8_t *q, const uint32_t *qn, int64_t q0, int64_t m,
                       const uint8_t *t, const uint32_t *tn, int64_t t0, int64_t n,
                       int64_t match, int64_t mismatch,
                       int64_t alpha, int64_t beta,
                       int64_t *Hrow, int64_t *Frow,
                       int64_t *score, int64_t *qend, int64_t *tend)
{
    int64_t best = 0, bi = -1, bj = -1;
    if (m <= 0 || n <= 0) {
        *score = 0; *qend = -1; *tend = -1;
        return;
    }
    for (int64_t j = 0; j < m; ++j) {
        Hrow[j] = 0;               /* H(-1, j) */
        Frow[j] = ORACLE_NEG_INF;  /* F(-1, j) */
    }
    for (int64_t i = 0; i < n; ++i) {
        const int ti = base_at(t, t0 + i);
        const int t_is_n = is_n(tn, t0 + i);
        int64_t h_left = 0;              /* H(i, -1) */
        int64_t e = ORACLE_NEG_INF;      /* E(i, -1) */
        int64_t h_diag = 0;              /* H(i-1, -1) */
        for (int64_t j = 0; j < m; ++j) {
            const int qj = base_at(q, q0 + j);
            const int64_t s_acgt = (ti == qj) ? match : mismatch;
            const int64_t s = (t_is_n || is_n(qn, q0 + j)) ? mismatch : s_acgt;
            /* E(i,j) from H(i,j-1) and E(i,j-1) */
            const int64_t e_open = h_left - alpha;
            const int64_t e_ext = e - beta;
            e = e_open > e_ext ? e_open : e_ext;
            /* F(i,j) from H(i-1,j) and F(i-1,j) */
            const int64_t f_open = Hrow[j] - alpha;
            const int64_t f_ext = Frow[j] - beta;
            const int64_t f = f_open > f_ext ? f_open : f_ext;
            /* H(i,j) */
            int64_t h = h_diag + s;
            if (e > h) h = e;
            if (f > h) h = f;
            if (h < 0) h = 0;
            h_diag = Hrow[j];   /* becomes H(i-1, j) for column j+1 */
            Hrow[j] = h;
            Frow[j] = f;
            h_left = h;
            if (h > best) {     /* strict: first maximum in row-major order */
                best = h; bi = i; bj = j;
            }
        }
    }
    *score = best;
    *qend = best > 0 ? bj : -1;
    *tend = best > 0 ? bi : -1;
}

typedef struct {
    const uint8_t *q, *t;
    const uint32_t *qn, *tn;
    const int64_t *q_off, *t_off;
    const int64_t *order;
    int64_t n;
    int64_t match, mismatch, alpha, beta;
    int64_t *score, *qend, *tend;
    int64_t next;            /* shared counter, taken under the mutex */
    pthread_mutex_t mu;
    int64_t max_m;
} job_t;

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    int64_t *Hrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(jb->max_m + 1));
    int64_t *Frow = (int64_t *)malloc(sizeof(int64_t) * (size_t)(jb->max_m + 1));
    if (!Hrow || !Frow) { free(Hrow); free(Frow); return (void *)1; }
    for (;;) {
        int64_t k0, k1;
        pthread_mutex_lock(&jb->mu);
        k0 = jb->next;
        /* hand out small runs of pairs; the first ones are the longest */
        k1 = k0 + 16 > jb->n ? jb->n : k0 + 16;
        jb->next = k1;
        pthread_mutex_unlock(&jb->mu);
        if (k0 >= jb->n) break;
        for (int64_t k = k0; k < k1; ++k) {
            const int64_t p = jb->order ? jb->order[k] : k;
            const int64_t q0 = jb->q_off[p], q1 = jb->q_off[p + 1];
            const int64_t t0 = jb->t_off[p], t1 = jb->t_off[p + 1];
            gotoh_pair(jb->q, jb->qn, q0, q1 - q0, jb->t, jb->tn, t0, t1 - t0,
                       jb->match, jb->mismatch, jb->alpha, jb->beta,
                       Hrow, Frow, &jb->score[p], &jb->qend[p], &jb->tend[p]);
        }
    }
    free(Hrow);
    free(Frow);
    return NULL;
}

/* Longest-first schedule: (cells, pair) records sorted by descending cell
 * count.  The comparator reads only its two records, so concurrent batch
 * calls from several host threads share no state. */
typedef struct {
    int64_t cells;
    int64_t pair;
} sched_t;

static int cmp_cells_desc(const void *a, const void *b)
{
    const int64_t x = ((const sched_t *)a)->cells;
    const int64_t y = ((const sched_t *)b)->cells;
    return (x < y) - (x > y);
}

/*
 * Align n_pairs pairs.  Offsets must be non-decreasing (the caller checks);
 * outputs are int64 arrays of length n_pairs.  nthreads <= 0 means 1.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_align_batch_n(const uint8_t *q_seqs, const uint32_t *q_nmask,
                         const int64_t *q_offsets,
                         const uint8_t *t_seqs, const uint32_t *t_nmask,
                         const int64_t *t_offsets,
                         int64_t n_pairs,
                         int64_t match, int64_t mismatch,
                         int64_t gap_open, int64_t gap_extend,
                         int64_t *out_score, int64_t *out_qend, int64_t *out_tend,
                         int nthreads)
{
    if (n_pairs <= 0) return 0;
    if (nthreads <= 0) nthreads = 1;
    if (nthreads > 256) nthreads = 256;

    job_t jb;
    memset(&jb, 0, sizeof jb);
    jb.q = q_seqs; jb.t = t_seqs; jb.q_off = q_offsets; jb.t_off = t_offsets;
    jb.qn = q_nmask; jb.tn = t_nmask;
    jb.n = n_pairs;
    jb.match = match; jb.mismatch = mismatch;
    jb.alpha = gap_open + gap_extend;   /* opening a gap of length 1 */
    jb.beta = gap_extend;               /* each further gap base */
    jb.score = out_score; jb.qend = out_qend; jb.tend = out_tend;
    pthread_mutex_init(&jb.mu, NULL);

    sched_t *sched = (sched_t *)malloc(sizeof(sched_t) * (size_t)n_pairs);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_pairs);
    if (!sched || !order) { free(sched); free(order); return -1; }
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int64_t m = q_offsets[p + 1] - q_offsets[p];
        const int64_t n = t_offsets[p + 1] - t_offsets[p];
        sched[p].cells = m * n;
        sched[p].pair = p;
        if (m > jb.max_m) jb.max_m = m;
    }
    qsort(sched, (size_t)n_pairs, sizeof(sched_t), cmp_cells_desc);
    for (int64_t k = 0; k < n_pairs; ++k) order[k] = sched[k].pair;
    free(sched);
    jb.order = order;

    int rc = 0;
    if (nthreads == 1) {
        if (worker(&jb) != NULL) rc = -1;
    } else {
        pthread_t th[256];
        int started = 0;
        for (int k = 0; k < nthreads; ++k) {
            if (pthread_create(&th[k], NULL, worker, &jb) != 0) break;
            ++started;
        }
        if (started == 0) { if (worker(&jb) != NULL) rc = -1; }
        for (int k = 0; k < started; ++k) {
            void *ret = NULL;
            pthread_join(th[k], &ret);
            if (ret != NULL) rc = -1;
        }
    }
    pthread_mutex_destroy(&jb.mu);
    free(order);
    return rc;
}

/* Without N masks: every base is A, C, G or T. */
int oracle_align_batch(const uint8_t *q_seqs, const int64_t *q_offsets,
                       const uint8_t *t_seqs, const int64_t *t_offsets,
                       int64_t n_pairs,
                       int64_t match, int64_t mismatch,
                       int64_t gap_open, int64_t gap_extend,
                       int64_t *out_score, int64_t *out_qend, int64_t *out_tend,
                       int nthreads)
{
    return oracle_align_batch_n(q_seqs, NULL, q_offsets, t_seqs, NULL, t_offsets, n_pairs,
                                match, mismatch, gap_open, gap_extend, out_score, out_qend,
                                out_tend, nthreads);
}

/* H value of one cell, for validity checks of an end position: returns
 * H(ti, qj) of the pair's table (0 <= ti < n, 0 <= qj < m), or -1 when the
 * indices are outside the table. */
int64_t oracle_cell_h(const uint8_t *q_seqs, int64_t q0, int64_t m,
                      const uint8_t *t_seqs, int64_t t0, int64_t n,
                      int64_t match, int64_t mismatch,
                      int64_t gap_open, int64_t gap_extend,
                      int64_t ti, int64_t qj)
{
    if (ti < 0 || qj < 0 || ti >= n || qj >= m) return -1;
    const int64_t alpha = gap_open + gap_extend, beta = gap_extend;
    int64_t *Hrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *Frow = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!Hrow || !Frow) { free(Hrow); free(Frow); return -2; }
    for (int64_t j = 0; j < m; ++j) { Hrow[j] = 0; Frow[j] = ORACLE_NEG_INF; }
    int64_t out = -1;
    for (int64_t i = 0; i <= ti; ++i) {
        const int tb = base_at(t_seqs, t0 + i);
        int64_t h_left = 0, e = ORACLE_NEG_INF, h_diag = 0;
        for (int64_t j = 0; j < m; ++j) {
            const int64_t s = (tb == base_at(q_seqs, q0 + j)) ? match : mismatch;
            const int64_t e1 = h_left - alpha, e2 = e - beta;
            e = e1 > e2 ? e1 : e2;
            const int64_t f1 = Hrow[j] - alpha, f2 = Frow[j] - beta;
            const int64_t f = f1 > f2 ? f1 : f2;
            int64_t h = h_diag + s;
            if (e > h) h = e;
            if (f > h) h = f;
            if (h < 0) h = 0;
            h_diag = Hrow[j];
            Hrow[j] = h;
            Frow[j] = f;
            h_left = h;
            if (i == ti && j == qj) out = h;
        }
    }
    free(Hrow);
    free(Frow);
    return out;
}
