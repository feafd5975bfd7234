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

/* Score of one (query, subject) pair.  q and d hold residue codes 0..a-1,
 * sm is the a x a substitution matrix row-major with rows indexed by the
 * query residue: SM(x, y) = sm[x * a + y].  Returns -1 on allocation failure. */
int64_t sw_oracle_pair(const int8_t* q, int64_t m, const int8_t* d, int64_t n,
                       const int8_t* sm, int64_t a, int64_t go, int64_t ge)
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
            int64_t H = Hdiag + (int64_t)sm[q[i - 1] * a + d[j - 1]];
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

/* ---------------- global and semi-global variants ----------------
 * The same recurrence without the local 0 in Eq. 1 and with gap borders:
 *   H[i][j] = max(H[i-1][j-1] + SM(Q[i], D[j]), E[i][j], F[i][j])
 *   E, F as in Eq. 2-3, E[i][0] = F[0][j] = minus infinity,
 *   H[i][0] = g(i)  and  H[0][j] = g(j) (global) or 0 (semi-global),
 * where g(k) = -(Go + (k-1) * min(Go, Ge)) for k >= 1 and g(0) = 0: the cost
 * the recurrence itself charges for a run of k gaps.
 *   mode 1, global: S = H[m][n], both sequences aligned end to end.
 *   mode 2, semi-global: S = max over j of H[m][j], the whole query aligned
 *   to any stretch of the subject (leading and trailing subject residues free).
 * mode 0 is the local score of sw_oracle_pair.  Returns INT64_MIN on
 * allocation failure. */
static int64_t gap_run(int64_t k, int64_t go, int64_t ge)
{
    return k <= 0 ? 0 : -(go + (k - 1) * (go < ge ? go : ge));
}

int64_t sw_oracle_pair_mode(const int8_t* q, int64_t m, const int8_t* d, int64_t n,
                            const int8_t* sm, int64_t a, int64_t go, int64_t ge, int64_t mode)
{
    if (mode == 0) return sw_oracle_pair(q, m, d, n, sm, a, go, ge);
    const int64_t NEG = INT64_MIN / 4;
    if (m <= 0) return mode == 1 ? gap_run(n, go, ge) : 0;
    if (n <= 0) return gap_run(m, go, ge);
    int64_t* Hup = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    int64_t* Fup = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!Hup || !Fup) { free(Hup); free(Fup); return INT64_MIN; }
    for (int64_t j = 0; j <= n; ++j) {
        Hup[j] = mode == 1 ? gap_run(j, go, ge) : 0;       /* row 0 */
        Fup[j] = NEG;
    }
    for (int64_t i = 1; i <= m; ++i) {
        int64_t Hleft = gap_run(i, go, ge);    /* H[i][0] */
        int64_t Eleft = NEG;                    /* E[i][0] */
        int64_t Hdiag = Hup[0];                 /* H[i-1][0] */
        Hup[0] = Hleft;
        for (int64_t j = 1; j <= n; ++j) {
            int64_t E = max2(Hleft - go, Eleft - ge);                 /* Eq. 2 */
            int64_t F = max2(Hup[j] - go, Fup[j] - ge);               /* Eq. 3 */
            int64_t H = Hdiag + (int64_t)sm[q[i - 1] * a + d[j - 1]];
            H = max2(H, E);
            H = max2(H, F);                                           /* Eq. 1 without the 0 */
            Hdiag = Hup[j];
            Hup[j] = H;
            Fup[j] = F;
            Hleft = H;
            Eleft = E;
        }
    }
    int64_t S = Hup[n];
    if (mode == 2)
        for (int64_t j = 0; j < n; ++j) S = max2(S, Hup[j]);
    free(Hup);
    free(Fup);
    return S;
}

/* ---------------- one query against many subjects, threads over subjects ---------------- */
typedef struct {
    const int8_t* q; int64_t m;
    const int8_t* res; const int64_t* offsets;
    const int64_t* idx; int64_t count;
    const int8_t* sm; int64_t a, go, ge, mode;
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
        int64_t v = sw_oracle_pair_mode(J->q, J->m, J->res + b, e - b, J->sm, J->a, J->go, J->ge, J->mode);
        if (J->mode == 0 ? v < 0 : v == INT64_MIN) J->failed = 1;
        J->out[k] = v;
    }
    return NULL;
}

/* Scores (mode 0 local, 1 global, 2 semi-global) of query q against subjects idx[0..count)
 * (all subjects 0..count if idx is NULL) of a database given as concatenated residues and offsets[n+1].
 * out[k] receives the score of subject idx[k].  nthreads <= 0 means 1.
 * Returns 0 on success, -1 on allocation or thread failure. */
int sw_oracle_scores(const int8_t* q, int64_t m, const int8_t* res, const int64_t* offsets,
                     const int64_t* idx, int64_t count, const int8_t* sm, int64_t a, int64_t go, int64_t ge,
                     int64_t mode, int32_t nthreads, int64_t* out)
{
    job_t J;
    memset(&J, 0, sizeof J);
    J.q = q; J.m = m; J.res = res; J.offsets = offsets; J.idx = idx; J.count = count;
    J.sm = sm; J.a = a; J.go = go; J.ge = ge; J.mode = mode; J.out = out;
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

/* ---------------- the alignment behind a score (traceback) ----------------
 * The optimal local alignment of q (m residues) against d (n residues): the
 * paper keeps alignments for the top-ranked subjects only and recovers them
 * by tracing back from the cell with the highest H (Sec. II-B).  Here the
 * full matrices H, E, F of Eq. 1-3 over (m+1) x (n+1) cells are kept (int32
 * storage, int64 arithmetic: every stored value lies in [-Go, S]), so the
 * inputs must be small.
 *
 * Several alignments may reach S.  This function returns the one fixed by:
 *   end cell: the first cell with H = S in row-major order (smallest i, then j);
 *   in H at (i, j): stop if H = 0 or i = 0 or j = 0 (the alignment starts
 *     after this cell); else the diagonal if H = H[i-1][j-1] + SM(q_i, d_j),
 *     else E if H = E[i][j], else F;
 *   in E at (i, j): d_j faces a gap ('D'); continue in H at (i, j-1) if
 *     E[i][j] = H[i][j-1] - Go (the gap opens there), else in E at (i, j-1);
 *   in F at (i, j): q_i faces a gap ('I'); continue in H at (i-1, j) if
 *     F[i][j] = H[i-1][j] - Go, else in F at (i-1, j);
 *   the diagonal aligns q_i with d_j ('M') and continues in H at (i-1, j-1).
 * out[0..4] = S, q_begin, q_end, s_begin, s_end (0-based residue indices,
 * end exclusive); ops[0..len) holds the operations from the first aligned
 * residue pair to the last.  Returns len, -1 on allocation failure, -2 if
 * cap < len. */
int64_t sw_oracle_align(const int8_t* q, int64_t m, const int8_t* d, int64_t n, const int8_t* sm, int64_t a,
                        int64_t go, int64_t ge, int64_t* out, char* ops, int64_t cap)
{
    for (int k = 0; k < 5; ++k) out[k] = 0;
    if (m <= 0 || n <= 0) return 0;
    const int64_t w = n + 1;
    int32_t* H = (int32_t*)calloc((size_t)((m + 1) * w), sizeof(int32_t));
    int32_t* E = (int32_t*)calloc((size_t)((m + 1) * w), sizeof(int32_t));
    int32_t* F = (int32_t*)calloc((size_t)((m + 1) * w), sizeof(int32_t));
    char* rev = (char*)malloc((size_t)(m + n + 1));
    if (!H || !E || !F || !rev) { free(H); free(E); free(F); free(rev); return -1; }
    int64_t S = 0, ei = 0, ej = 0;
    for (int64_t i = 1; i <= m; ++i) {
        for (int64_t j = 1; j <= n; ++j) {
            const int64_t e = max2((int64_t)H[i * w + j - 1] - go, (int64_t)E[i * w + j - 1] - ge);      /* Eq. 2 */
            const int64_t f = max2((int64_t)H[(i - 1) * w + j] - go, (int64_t)F[(i - 1) * w + j] - ge);  /* Eq. 3 */
            int64_t h = (int64_t)H[(i - 1) * w + j - 1] + sm[q[i - 1] * a + d[j - 1]];
            h = max2(max2(h, e), max2(f, 0));                                                          /* Eq. 1 */
            E[i * w + j] = (int32_t)e;
            F[i * w + j] = (int32_t)f;
            H[i * w + j] = (int32_t)h;
            if (h > S) { S = h; ei = i; ej = j; }
        }
    }
    int64_t len = 0, i = ei, j = ej;
    int state = 0;                  /* 0: H, 1: E, 2: F */
    while (S > 0) {
        if (state == 0) {
            const int64_t h = H[i * w + j];
            if (h == 0 || i == 0 || j == 0) break;
            if (h == (int64_t)H[(i - 1) * w + j - 1] + sm[q[i - 1] * a + d[j - 1]]) {
                rev[len++] = 'M';
                --i; --j;
            } else if (h == E[i * w + j]) {
                state = 1;
            } else {
                state = 2;
            }
        } else if (i < 1 || j < 1 || len >= m + n) {
            break;                  /* unreachable for a consistent trace; guards the walk */
        } else if (state == 1) {
            rev[len++] = 'D';
            if ((int64_t)E[i * w + j] == (int64_t)H[i * w + j - 1] - go) state = 0;
            --j;
        } else {
            rev[len++] = 'I';
            if ((int64_t)F[i * w + j] == (int64_t)H[(i - 1) * w + j] - go) state = 0;
            --i;
        }
    }
    free(H); free(E); free(F);
    if (len > cap) { free(rev); return -2; }
    for (int64_t k = 0; k < len; ++k) ops[k] = rev[len - 1 - k];
    free(rev);
    out[0] = S;
    out[1] = S > 0 ? i : 0;
    out[2] = ei;
    out[3] = S > 0 ? j : 0;
    out[4] = ej;
    return len;
}
