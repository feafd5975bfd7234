/*
 * CPU oracle for Smith-Waterman local alignment with Gotoh affine gaps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and never calls it.
 *
 * What it computes (Sec. II-B, Eq. 1-3 of the paper):
 *   H[i][j] = max(0, H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])   (Eq. 1)
 *   E[i][j] = max(H[i][j-1] - Go, E[i][j-1] - Ge)                        (Eq. 2)
 *   F[i][j] = max(H[i-1][j] - Go, F[i-1][j] - Ge)                        (Eq. 3)
 * with H = E = F = 0 whenever i = 0 or j = 0, and the score S is the largest
 * entry of H (0 for an empty sequence).  Only the score is wanted, so the
 * matrices are kept one row at a time (linear space, Sec. II-B last paragraph).
 *
 * Arithmetic is in int64 so that no intermediate can overflow for any
 * int32-range input; the paper's application uses int32 cells (Sec. III-B),
 * whose scores for protein inputs stay far below 2^31, so both agree.
 *
 * Plain C, scalar, no intrinsics, no blocking: each cell follows the three
 * equations above in the paper's notation.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* Score of one (query, subject) pair.  q and d hold residue codes 0..19,
 * sm is the 20x20 substitution matrix row-major with rows indexed by the
 * query residue: SM(a, b) = sm[a * 20 + b].  Returns -1 on allocation failure. */
int64_t sw_oracle_pair(const int8_t* q, int64_t m, const int8_t* d, int64_t n,
                       const int8_t* sm, int64_t go, int64_t ge)
{
    if (m <= 0 || n <= 0) return 0;
    /* Hup[j] = H[i-1][j] and Fup[j] = F[i-1][j] for the row above; row 0 is zero. */
    int64_t* Hup = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* Fup = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!Hup || !Fup) { free(Hup); free(Fup); return -1; }
    int64_t S = 0;
    for (int64_t i = 1; i <= m; ++i) {
        int64_t Hleft = 0;      /* H[i][0] */
        int64_t Eleft = 0;      /* E[i][0] */
        int64_t Hdiag = 0;      /* H[i-1][0] */
        for (int64_t j = 1; j <= n; ++j) {
            int64_t E = max2(Hleft - go, Eleft - ge);                 /* Eq. 2 */
            int64_t F = max2(Hup[j] - go, Fup[j] - ge);               /* Eq. 3 */
            int64_t H = Hdiag + (int64_t)sm[q[i - 1] * 20 + d[j - 1]];
            H = max2(H, E);
            H = max2(H, F);
            H = max2(H, 0);                                           /* Eq. 1 */
            if (H > S) S = H;
            Hdiag = Hup[j];     /* H[i-1][j] is the upper-left neighbour of (i, j+1) */
            Hup[j] = H;
            Fup[j] = F;
            Hleft = H;
            Eleft = E;
        }
    }
    free(Hup);
    free(Fup);
    return S;
}

/* ---------------- one query against many subjects, threads over subjects ---------------- */
typedef struct {
    const int8_t* q; int64_t m;
    const int8_t* res; const int64_t* offsets;
    const int64_t* idx; int64_t count;
    const int8_t* sm; int64_t go, ge;
    int64_t* out;
    int64_t next;               /* shared work counter */
    pthread_mutex_t lock;
    int failed;
} job_t;

static void* worker(void* arg)
{
    job_t* J = (job_t*)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t k = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (k >= J->count) break;
        int64_t s = J->idx ? J->idx[k] : k;
        int64_t b = J->offsets[s], e = J->offsets[s + 1];
        int64_t v = sw_oracle_pair(J->q, J->m, J->res + b, e - b, J->sm, J->go, J->ge);
        if (v < 0) J->failed = 1;
        J->out[k] = v;
    }
    return NULL;
}

/* Scores of query q against subjects idx[0..count) (all subjects 0..count if idx
 * is NULL) of a database given as concatenated residues and offsets[n+1].
 * out[k] receives the score of subject idx[k].  nthreads <= 0 means 1.
 * Returns 0 on success, -1 on allocation or thread failure. */
int sw_oracle_scores(const int8_t* q, int64_t m, const int8_t* res, const int64_t* offsets,
                     const int64_t* idx, int64_t count, const int8_t* sm, int64_t go, int64_t ge,
                     int32_t nthreads, int64_t* out)
{
    job_t J;
    memset(&J, 0, sizeof J);
    J.q = q; J.m = m; J.res = res; J.offsets = offsets; J.idx = idx; J.count = count;
    J.sm = sm; J.go = go; J.ge = ge; J.out = out;
    pthread_mutex_init(&J.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, worker, &J) != 0) { J.failed = 1; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.failed ? -1 : 0;
}
