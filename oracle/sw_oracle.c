/*
 * Oracle for Smith-Waterman protein database search -- TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain, slow, obviously correct CPU reference that the GPU path is
 * checked against.  Only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg may load it; the library that users call never does.
 *
 * What it computes (paper, Section 2, Eqs. 1-3 and the paragraph after them):
 *
 *   H[i][j] = max{ 0, H[i-1][j-1] + SM(S1[i], S2[j]), E[i][j], F[i][j] }      (Eq. 1)
 *   E[i][j] = max{ H[i][j-1] - Goe, E[i][j-1] - Ge }                          (Eq. 2)
 *   F[i][j] = max{ H[i-1][j] - Goe, F[i-1][j] - Ge }                          (Eq. 3)
 *
 * for 1 <= i <= m (query S1) and 1 <= j <= n (database sequence S2), with H, E and F
 * set to 0 whenever i = 0 or j = 0.  Goe is the sum of the gap-open and gap-extend
 * penalties and Ge is the gap-extend penalty.  The alignment score is the largest
 * entry of H, which is never negative.
 *
 * Arithmetic is plain int32, row by row, with nothing blocked, fused or vectorised.
 * SM is indexed as matrix[S1[i] * alphabet + S2[j]] (the query residue picks the row).
 *
 * A database search (Section 4: the SW stage) is just this score for the query
 * against every sequence; sequences are split statically across POSIX threads.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int32_t max2(int32_t a, int32_t b) { return a > b ? a : b; }

/*
 * Score of one query/sequence pair.  `ef_border` is the value E and F take on row 0
 * and column 0: the paper uses 0; passing a very negative value gives the textbook
 * "minus infinity" border so that a test can show both readings agree.
 * Returns -1 on allocation failure.
 */
int32_t swo_score_border(const uint8_t *s1, int32_t m, const uint8_t *s2, int32_t n,
                         const int32_t *sm, int32_t alphabet, int32_t gap_open,
                         int32_t gap_extend, int32_t ef_border)
{
    if (m <= 0 || n <= 0) return 0;
    const int32_t goe = gap_open + gap_extend;
    const int32_t ge = gap_extend;

    /* previous and current rows of H, E and F, each with the j = 0 column */
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)(n + 1));
    if (!buf) return -1;
    int32_t *h_prev = buf, *e_prev = buf + (n + 1), *f_prev = buf + 2 * (n + 1);
    int32_t *h_cur = buf + 3 * (n + 1), *e_cur = buf + 4 * (n + 1), *f_cur = buf + 5 * (n + 1);

    /* row i = 0 */
    for (int32_t j = 0; j <= n; ++j) {
        h_prev[j] = 0;
        e_prev[j] = ef_border;
        f_prev[j] = ef_border;
    }
    int32_t best = 0;
    for (int32_t i = 1; i <= m; ++i) {
        /* column j = 0 */
        h_cur[0] = 0;
        e_cur[0] = ef_border;
        f_cur[0] = ef_border;
        const int32_t *row = sm + (size_t)s1[i - 1] * alphabet;
        for (int32_t j = 1; j <= n; ++j) {
            int32_t e = max2(h_cur[j - 1] - goe, e_cur[j - 1] - ge);        /* Eq. 2 */
            int32_t f = max2(h_prev[j] - goe, f_prev[j] - ge);              /* Eq. 3 */
            int32_t h = max2(max2(0, h_prev[j - 1] + row[s2[j - 1]]),
                             max2(e, f));                                    /* Eq. 1 */
            e_cur[j] = e;
            f_cur[j] = f;
            h_cur[j] = h;
            best = max2(best, h);
        }
        int32_t *t;
        t = h_prev; h_prev = h_cur; h_cur = t;
        t = e_prev; e_prev = e_cur; e_cur = t;
        t = f_prev; f_prev = f_cur; f_cur = t;
    }
    free(buf);
    return best;
}

int32_t swo_score(const uint8_t *s1, int32_t m, const uint8_t *s2, int32_t n,
                  const int32_t *sm, int32_t alphabet, int32_t gap_open, int32_t gap_extend)
{
    return swo_score_border(s1, m, s2, n, sm, alphabet, gap_open, gap_extend, 0);
}

typedef struct {
    const uint8_t *query;
    int32_t m;
    const uint8_t *residues;
    const int64_t *offsets;
    const int64_t *index; /* optional subset of sequences; NULL means all */
    int64_t begin, end;
    const int32_t *sm;
    int32_t alphabet, gap_open, gap_extend;
    int32_t *scores;
    int failed;
} swo_job;

static void *swo_worker(void *arg)
{
    swo_job *job = (swo_job *)arg;
    for (int64_t t = job->begin; t < job->end; ++t) {
        int64_t k = job->index ? job->index[t] : t;
        const uint8_t *s2 = job->residues + job->offsets[k];
        int32_t n = (int32_t)(job->offsets[k + 1] - job->offsets[k]);
        int32_t s = swo_score(job->query, job->m, s2, n, job->sm, job->alphabet,
                              job->gap_open, job->gap_extend);
        if (s < 0) job->failed = 1;
        job->scores[t] = s;
    }
    return NULL;
}

/*
 * Score the query against sequences of a database given as concatenated residues
 * plus n_seqs+1 offsets.  If `index` is non-NULL, only sequences index[0..count) are
 * scored and scores[t] belongs to index[t]; otherwise count must equal n_seqs.
 * Work is split statically into `n_threads` contiguous ranges.
 * Returns 0 on success, -1 on failure.
 */
int swo_search(const uint8_t *query, int32_t m, const uint8_t *residues,
               const int64_t *offsets, const int64_t *index, int64_t count,
               const int32_t *sm, int32_t alphabet, int32_t gap_open, int32_t gap_extend,
               int32_t *scores, int32_t n_threads)
{
    if (count <= 0) return 0;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > count) n_threads = (int32_t)count;
    swo_job *jobs = (swo_job *)calloc((size_t)n_threads, sizeof(swo_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) { free(jobs); free(tids); return -1; }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 0; t < n_threads; ++t) {
        swo_job *j = &jobs[t];
        j->query = query; j->m = m; j->residues = residues; j->offsets = offsets;
        j->index = index;
        j->begin = count * t / n_threads;
        j->end = count * (t + 1) / n_threads;
        j->sm = sm; j->alphabet = alphabet; j->gap_open = gap_open; j->gap_extend = gap_extend;
        j->scores = scores;
        if (pthread_create(&tids[t], NULL, swo_worker, j) != 0) { rc = -1; break; }
        ++started;
    }
    for (int32_t t = 0; t < started; ++t) {
        pthread_join(tids[t], NULL);
        if (jobs[t].failed) rc = -1;
    }
    free(jobs);
    free(tids);
    return rc;
}
