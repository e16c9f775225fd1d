/*
 * CPU oracle for score-only pairwise alignment (Gotoh affine-gap dynamic
 * program) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library never links it, never
 * calls it and shares no code with it.
 *
 * Everything here is the plain textbook definition, computed in 64-bit
 * integers, one matrix row at a time (linear memory, quadratic time; the
 * paper's "Traceback" paragraph of section 2.1 notes score-only needs only
 * linear space).  No blocking, no vectorisation, no reordering.
 *
 * Notation (paper, section 2.1 "Sequence Alignment"):
 *   Q = q_1..q_m  (rows, i),  S = s_1..s_n  (columns, j)
 *   H(i,j) = max{ H(i-1,j-1) + sigma(q_i,s_j), E(i,j), F(i,j), nu }   Eq. (1)
 *   E(i,j) = max{ E(i-1,j) - beta, H(i-1,j) - alpha }                 Eq. (4)
 *   F(i,j) = max{ F(i,j-1) - beta, H(i,j-1) - alpha }                 Eq. (5)
 *   A gap of length k costs alpha + (k-1)*beta; linear gaps are alpha == beta
 *   (Eq. (2),(3) are the alpha == beta case, because H >= E and H >= F).
 *
 * Modes ("Local / Global / Semi-global Alignments" paragraphs, section 2.1):
 *   global      nu = -inf; H(i,0) = -alpha - beta(i-1), H(0,j) likewise,
 *               H(0,0) = 0; result H(m,n).
 *   local       nu = 0; H(i,0) = H(0,j) = 0; result max over every cell.
 *   semi-global initialisation as local, nu = -inf (reading: the paper
 *               shares only the initialisation with local; nu = 0 would make
 *               mismatching prefixes free, which is not a free end gap);
 *               result = max over the last row and the last column,
 *               including the boundary cells H(m,0) and H(0,n).
 *   In every mode E(0,j) = F(i,0) = -inf; the paper's E(i,0), F(0,j) values
 *   are never read by a cell with i,j >= 1.
 *
 * Banded variant (not in the paper; the learned-band extension): a cell
 * (i,j), boundary cells included, exists only when L <= j-i <= U with
 *   L = min(0, n-m) - w,  U = max(0, n-m) + w,  w >= 0;
 * cells outside are -inf in H, E and F.  The result is taken as in the full
 * mode over existing cells only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_NEG_INF (-(((int64_t)1) << 60))

enum { ORACLE_GLOBAL = 0, ORACLE_SEMIGLOBAL = 1, ORACLE_LOCAL = 2 };

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* Initial value of the boundary cell H(i,0) (or H(0,j) with i := j). */
static int64_t boundary_h(int64_t i, int32_t mode, int64_t alpha, int64_t beta) {
    if (i == 0) return 0;
    if (mode == ORACLE_GLOBAL) return -alpha - beta * (i - 1);
    return 0;
}

/* Score of one pair, restricted to the band [lo, hi] of diagonals j-i.
 * The full problem is lo = -m, hi = n. */
static int64_t align_band(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                          const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                          int32_t mode, int64_t lo, int64_t hi) {
    const int64_t nu = (mode == ORACLE_LOCAL) ? 0 : ORACLE_NEG_INF;
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1)); /* row i-1, then row i */
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1)); /* E(i-1,j), then E(i,j) */
    int64_t best = ORACLE_NEG_INF;
    int64_t j, i;

    /* row 0 */
    for (j = 0; j <= n; ++j) {
        int in_band = (j - 0 >= lo) && (j - 0 <= hi);
        H[j] = in_band ? boundary_h(j, mode, alpha, beta) : ORACLE_NEG_INF;
        E[j] = ORACLE_NEG_INF;
    }
    if (mode == ORACLE_LOCAL) {
        for (j = 0; j <= n; ++j) best = max2(best, H[j]);
    }
    if (mode == ORACLE_SEMIGLOBAL) {
        best = max2(best, H[n]); /* H(0,n): last column, row 0 */
        if (m == 0)
            for (j = 0; j <= n; ++j) best = max2(best, H[j]); /* row 0 is the last row */
    }

    for (i = 1; i <= m; ++i) {
        int64_t diag = H[0];                       /* H(i-1, 0) */
        int64_t F = ORACLE_NEG_INF;                /* F(i, 0) */
        int in_band0 = (0 - i >= lo) && (0 - i <= hi);
        H[0] = in_band0 ? boundary_h(i, mode, alpha, beta) : ORACLE_NEG_INF;
        for (j = 1; j <= n; ++j) {
            int64_t up = H[j]; /* H(i-1, j) */
            int64_t h;
            if (j - i < lo || j - i > hi) {
                E[j] = ORACLE_NEG_INF;
                F = ORACLE_NEG_INF;
                h = ORACLE_NEG_INF;
            } else {
                int64_t sigma = subst[(int32_t)q[i - 1] * asz + (int32_t)s[j - 1]];
                int64_t e = max2(E[j] - beta, up - alpha);
                int64_t f = max2(F - beta, H[j - 1] - alpha);
                h = diag + sigma;
                h = max2(h, e);
                h = max2(h, f);
                h = max2(h, nu);
                /* keep -inf from drifting upwards out of the sentinel range */
                if (e < ORACLE_NEG_INF) e = ORACLE_NEG_INF;
                if (f < ORACLE_NEG_INF) f = ORACLE_NEG_INF;
                if (h < ORACLE_NEG_INF) h = ORACLE_NEG_INF;
                E[j] = e;
                F = f;
            }
            diag = up;
            H[j] = h;
            if (mode == ORACLE_LOCAL) best = max2(best, h);
        }
        if (mode == ORACLE_LOCAL) best = max2(best, H[0]);
        if (mode == ORACLE_SEMIGLOBAL) best = max2(best, H[n]); /* last column, row i */
    }
    if (mode == ORACLE_SEMIGLOBAL && m > 0)
        for (j = 0; j <= n; ++j) best = max2(best, H[j]); /* last row */
    if (mode == ORACLE_GLOBAL) best = H[n];
    free(H);
    free(E);
    return best;
}

int64_t oracle_align_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                          const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                          int32_t mode) {
    return align_band(q, m, s, n, subst, asz, alpha, beta, mode, -m, n);
}

int64_t oracle_banded_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                           const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                           int32_t mode, int64_t w) {
    int64_t lo = (n - m < 0 ? n - m : 0) - w;
    int64_t hi = (n - m > 0 ? n - m : 0) + w;
    return align_band(q, m, s, n, subst, asz, alpha, beta, mode, lo, hi);
}

/* Score restricted to the diagonals lo <= j-i <= hi (explicit limits). */
int64_t oracle_diag_band_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                              const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                              int32_t mode, int64_t lo, int64_t hi) {
    return align_band(q, m, s, n, subst, asz, alpha, beta, mode, lo, hi);
}

/* ---- threaded batch driver: pairs are independent, split them over threads ---- */

typedef struct {
    const uint8_t *sa, *sb;
    const int64_t *oa, *ob;
    const int64_t *band_w; /* NULL = full DP */
    const int64_t *band_lo, *band_hi; /* explicit diagonal limits (overrides band_w) */
    int64_t n_pairs;
    const int8_t *subst;
    int32_t asz, mode;
    int64_t alpha, beta;
    int64_t *out;
    int64_t next; /* shared work counter */
    pthread_mutex_t lock;
} batch_job;

static void *batch_worker(void *arg) {
    batch_job *job = (batch_job *)arg;
    for (;;) {
        int64_t p0, p1, p;
        pthread_mutex_lock(&job->lock);
        p0 = job->next;
        job->next += 16;
        pthread_mutex_unlock(&job->lock);
        if (p0 >= job->n_pairs) break;
        p1 = p0 + 16 < job->n_pairs ? p0 + 16 : job->n_pairs;
        for (p = p0; p < p1; ++p) {
            const uint8_t *q = job->sa + job->oa[p];
            const uint8_t *s = job->sb + job->ob[p];
            int64_t m = job->oa[p + 1] - job->oa[p];
            int64_t n = job->ob[p + 1] - job->ob[p];
            if (job->band_lo)
                job->out[p] = oracle_diag_band_pair(q, m, s, n, job->subst, job->asz, job->alpha,
                                                    job->beta, job->mode, job->band_lo[p],
                                                    job->band_hi[p]);
            else if (job->band_w)
                job->out[p] = oracle_banded_pair(q, m, s, n, job->subst, job->asz, job->alpha,
                                                 job->beta, job->mode, job->band_w[p]);
            else
                job->out[p] = oracle_align_pair(q, m, s, n, job->subst, job->asz, job->alpha,
                                                job->beta, job->mode);
        }
    }
    return NULL;
}

static void run_batch(batch_job *job, int32_t nthreads) {
    pthread_t *th;
    int32_t t;
    if (nthreads < 1) nthreads = 1;
    th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    pthread_mutex_init(&job->lock, NULL);
    job->next = 0;
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, batch_worker, job);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job->lock);
    free(th);
}

void oracle_align_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                        const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                        int64_t alpha, int64_t beta, int32_t mode, int32_t nthreads, int64_t *out) {
    batch_job job;
    memset(&job, 0, sizeof(job));
    job.sa = seqs_a; job.sb = seqs_b; job.oa = offs_a; job.ob = offs_b;
    job.band_w = NULL; job.n_pairs = n_pairs; job.subst = subst; job.asz = asz;
    job.mode = mode; job.alpha = alpha; job.beta = beta; job.out = out;
    run_batch(&job, nthreads);
}

void oracle_banded_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                         const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                         int64_t alpha, int64_t beta, int32_t mode, const int64_t *band_w,
                         int32_t nthreads, int64_t *out) {
    batch_job job;
    memset(&job, 0, sizeof(job));
    job.sa = seqs_a; job.sb = seqs_b; job.oa = offs_a; job.ob = offs_b;
    job.band_w = band_w; job.n_pairs = n_pairs; job.subst = subst; job.asz = asz;
    job.mode = mode; job.alpha = alpha; job.beta = beta; job.out = out;
    run_batch(&job, nthreads);
}

void oracle_diag_band_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                            const int64_t *offs_b, int64_t n_pairs, const int8_t *subst,
                            int32_t asz, int64_t alpha, int64_t beta, int32_t mode,
                            const int64_t *lo, const int64_t *hi, int32_t nthreads, int64_t *out) {
    batch_job job;
    memset(&job, 0, sizeof(job));
    job.sa = seqs_a; job.sb = seqs_b; job.oa = offs_a; job.ob = offs_b;
    job.band_lo = lo; job.band_hi = hi; job.n_pairs = n_pairs; job.subst = subst; job.asz = asz;
    job.mode = mode; job.alpha = alpha; job.beta = beta; job.out = out;
    run_batch(&job, nthreads);
}

/* ---- alignments and traceback ("Traceback" paragraph of section 2.1) ----
 *
 * An alignment is a string of columns: 'M' puts q_i against s_j (match or
 * mismatch), 'I' puts q_i against a gap (a step down a matrix column), 'D'
 * puts s_j against a gap (a step along a matrix row).  It covers the
 * substrings Q[a0..a1) and S[b0..b1), span = {a0, a1, b0, b1}.  Its score is
 * the definition itself: sigma summed over the 'M' columns, minus
 * alpha + (k-1)*beta for every maximal run of k equal gap columns ('I' runs
 * and 'D' runs are separate runs, Eq. (4),(5)).  Which spans a mode admits
 * (the mode paragraphs of section 2.1):
 *   global       the whole of both sequences: a0 = b0 = 0, a1 = m, b1 = n;
 *   semi-global  free end gaps: the part cut off in front is a prefix of one
 *                sequence only (a0 == 0 or b0 == 0), likewise at the end
 *                (a1 == m or b1 == n);
 *   local        any substrings (the empty alignment included).
 * oracle_alignment_score returns ORACLE_INVALID when the columns do not
 * consume exactly the span or the mode does not admit the span.
 */
#define ORACLE_INVALID INT64_MIN

int64_t oracle_alignment_score(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                               const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                               int32_t mode, const uint8_t *ops, int64_t n_ops,
                               const int32_t *span) {
    int64_t a0 = span[0], a1 = span[1], b0 = span[2], b1 = span[3];
    int64_t i = a0, j = b0, k, score = 0;
    uint8_t prev = 0;
    if (a0 < 0 || a0 > a1 || a1 > m || b0 < 0 || b0 > b1 || b1 > n || n_ops < 0) return ORACLE_INVALID;
    if (mode == ORACLE_GLOBAL && (a0 != 0 || b0 != 0 || a1 != m || b1 != n)) return ORACLE_INVALID;
    if (mode == ORACLE_SEMIGLOBAL && ((a0 != 0 && b0 != 0) || (a1 != m && b1 != n))) return ORACLE_INVALID;
    for (k = 0; k < n_ops; ++k) {
        uint8_t op = ops[k];
        if (op == 'M') {
            if (i >= a1 || j >= b1) return ORACLE_INVALID;
            score += subst[(int32_t)q[i] * asz + (int32_t)s[j]];
            ++i;
            ++j;
        } else if (op == 'I' || op == 'D') {
            if (op == 'I' && i >= a1) return ORACLE_INVALID;
            if (op == 'D' && j >= b1) return ORACLE_INVALID;
            score -= (prev == op) ? beta : alpha; /* a new run opens, or the run goes on */
            if (op == 'I') ++i; else ++j;
        } else {
            return ORACLE_INVALID;
        }
        prev = op;
    }
    if (i != a1 || j != b1) return ORACLE_INVALID;
    return score;
}

/* One optimal alignment: the full matrices H, E, F of Eq. (1),(4),(5) in the
 * mode's initialisation (quadratic memory: for small pairs only), then a walk
 * back from the mode's result cell through the predecessor each value was
 * taken from.  Ties go to the diagonal, then E, then F; a gap value taken
 * equally from an open and an extension goes to the open.  ops_out receives
 * the columns from the first to the last (at most m + n), span_out =
 * {n_ops, a0, a1, b0, b1}.  Returns the optimal score. */
int64_t oracle_traceback_pair(const uint8_t *q, int64_t m, const uint8_t *s, int64_t n,
                              const int8_t *subst, int32_t asz, int64_t alpha, int64_t beta,
                              int32_t mode, uint8_t *ops_out, int32_t *span_out) {
    const int64_t W = n + 1;
    const int64_t nu = (mode == ORACLE_LOCAL) ? 0 : ORACLE_NEG_INF;
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
    int64_t *E = (int64_t *)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)((m + 1) * W));
    uint8_t *rev = (uint8_t *)malloc((size_t)(m + n + 1));
    int64_t i, j, best, bi, bj, k = 0, len;
    int state = 0; /* 0: H, 1: E (vertical gap), 2: F (horizontal gap) */
#define AT(X, r, c) X[(r) * W + (c)]
    for (i = 0; i <= m; ++i)
        for (j = 0; j <= n; ++j) {
            AT(E, i, j) = ORACLE_NEG_INF;
            AT(F, i, j) = ORACLE_NEG_INF;
            if (i == 0) AT(H, i, j) = boundary_h(j, mode, alpha, beta);
            else if (j == 0) AT(H, i, j) = boundary_h(i, mode, alpha, beta);
        }
    for (i = 1; i <= m; ++i)
        for (j = 1; j <= n; ++j) {
            int64_t sigma = subst[(int32_t)q[i - 1] * asz + (int32_t)s[j - 1]];
            int64_t e = max2(AT(E, i - 1, j) - beta, AT(H, i - 1, j) - alpha);
            int64_t f = max2(AT(F, i, j - 1) - beta, AT(H, i, j - 1) - alpha);
            int64_t h = max2(max2(AT(H, i - 1, j - 1) + sigma, e), max2(f, nu));
            AT(E, i, j) = e < ORACLE_NEG_INF ? ORACLE_NEG_INF : e;
            AT(F, i, j) = f < ORACLE_NEG_INF ? ORACLE_NEG_INF : f;
            AT(H, i, j) = h < ORACLE_NEG_INF ? ORACLE_NEG_INF : h;
        }
    /* the result cell of the mode (first in row-major order among equals) */
    if (mode == ORACLE_GLOBAL) {
        bi = m; bj = n; best = AT(H, m, n);
    } else if (mode == ORACLE_LOCAL) {
        bi = 0; bj = 0; best = 0;
        for (i = 0; i <= m; ++i)
            for (j = 0; j <= n; ++j)
                if (AT(H, i, j) > best) { best = AT(H, i, j); bi = i; bj = j; }
    } else {
        bi = -1; bj = -1; best = ORACLE_NEG_INF;
        for (i = 0; i <= m; ++i)
            for (j = 0; j <= n; ++j)
                if ((i == m || j == n) && AT(H, i, j) > best) { best = AT(H, i, j); bi = i; bj = j; }
    }
    span_out[2] = (int32_t)bi;
    span_out[4] = (int32_t)bj;
    i = bi;
    j = bj;
    for (;;) {
        if (state == 0) {
            if (i == 0 && j == 0) break;
            if (j == 0 || i == 0) {
                /* the boundary: a gap run from the corner (global) or a free start */
                if (mode != ORACLE_GLOBAL) break;
                while (i > 0) { rev[k++] = 'I'; --i; }
                while (j > 0) { rev[k++] = 'D'; --j; }
                break;
            }
            {
                int64_t h = AT(H, i, j);
                int64_t sigma = subst[(int32_t)q[i - 1] * asz + (int32_t)s[j - 1]];
                if (mode == ORACLE_LOCAL && h == 0) break; /* nu = 0: the alignment starts here */
                if (h == AT(H, i - 1, j - 1) + sigma) {
                    rev[k++] = 'M';
                    --i;
                    --j;
                } else if (h == AT(E, i, j)) {
                    state = 1;
                } else {
                    state = 2;
                }
            }
        } else if (state == 1) {
            int64_t e = AT(E, i, j);
            rev[k++] = 'I';
            state = (e == AT(H, i - 1, j) - alpha) ? 0 : 1;
            --i;
        } else {
            int64_t f = AT(F, i, j);
            rev[k++] = 'D';
            state = (f == AT(H, i, j - 1) - alpha) ? 0 : 2;
            --j;
        }
    }
#undef AT
    span_out[1] = (int32_t)i;
    span_out[3] = (int32_t)j;
    span_out[0] = (int32_t)k;
    for (len = 0; len < k; ++len) ops_out[len] = rev[k - 1 - len];
    free(H);
    free(E);
    free(F);
    free(rev);
    return best;
}

/* ---- threaded batch drivers of the two functions above ---- */

typedef struct {
    const uint8_t *sa, *sb;
    const int64_t *oa, *ob;
    int64_t n_pairs;
    const int8_t *subst;
    int32_t asz, mode;
    int64_t alpha, beta;
    uint8_t *ops;          /* pair p at (oa[p] - oa[0]) + (ob[p] - ob[0]) */
    int32_t *span;         /* [n_pairs][5] */
    int64_t *out;
    int traceback;         /* 1: oracle_traceback_pair, 0: oracle_alignment_score */
    int64_t next;
    pthread_mutex_t lock;
} aln_job;

static void *aln_worker(void *arg) {
    aln_job *job = (aln_job *)arg;
    for (;;) {
        int64_t p0, p1, p;
        pthread_mutex_lock(&job->lock);
        p0 = job->next;
        job->next += 8;
        pthread_mutex_unlock(&job->lock);
        if (p0 >= job->n_pairs) break;
        p1 = p0 + 8 < job->n_pairs ? p0 + 8 : job->n_pairs;
        for (p = p0; p < p1; ++p) {
            const uint8_t *q = job->sa + job->oa[p];
            const uint8_t *s = job->sb + job->ob[p];
            int64_t m = job->oa[p + 1] - job->oa[p];
            int64_t n = job->ob[p + 1] - job->ob[p];
            uint8_t *ops = job->ops + (job->oa[p] - job->oa[0]) + (job->ob[p] - job->ob[0]);
            int32_t *sp = job->span + 5 * p;
            if (job->traceback) {
                job->out[p] = oracle_traceback_pair(q, m, s, n, job->subst, job->asz, job->alpha,
                                                    job->beta, job->mode, ops, sp);
            } else {
                int32_t span4[4];
                span4[0] = sp[1]; span4[1] = sp[2]; span4[2] = sp[3]; span4[3] = sp[4];
                job->out[p] = (sp[0] < 0 || sp[0] > m + n)
                                  ? ORACLE_INVALID
                                  : oracle_alignment_score(q, m, s, n, job->subst, job->asz, job->alpha,
                                                           job->beta, job->mode, ops, sp[0], span4);
            }
        }
    }
    return NULL;
}

static void run_aln(aln_job *job, int32_t nthreads) {
    pthread_t *th;
    int32_t t;
    if (nthreads < 1) nthreads = 1;
    th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    pthread_mutex_init(&job->lock, NULL);
    job->next = 0;
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, aln_worker, job);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job->lock);
    free(th);
}

/* span layout of both batch functions: [n_pairs][5] = n_ops, a0, a1, b0, b1 */
void oracle_traceback_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                            const int64_t *offs_b, int64_t n_pairs, const int8_t *subst, int32_t asz,
                            int64_t alpha, int64_t beta, int32_t mode, int32_t nthreads,
                            uint8_t *ops, int32_t *span, int64_t *out) {
    aln_job job;
    memset(&job, 0, sizeof(job));
    job.sa = seqs_a; job.sb = seqs_b; job.oa = offs_a; job.ob = offs_b; job.n_pairs = n_pairs;
    job.subst = subst; job.asz = asz; job.mode = mode; job.alpha = alpha; job.beta = beta;
    job.ops = ops; job.span = span; job.out = out; job.traceback = 1;
    run_aln(&job, nthreads);
}

void oracle_alignment_score_batch(const uint8_t *seqs_a, const int64_t *offs_a, const uint8_t *seqs_b,
                                  const int64_t *offs_b, int64_t n_pairs, const int8_t *subst,
                                  int32_t asz, int64_t alpha, int64_t beta, int32_t mode,
                                  int32_t nthreads, const uint8_t *ops, const int32_t *span,
                                  int64_t *out) {
    aln_job job;
    memset(&job, 0, sizeof(job));
    job.sa = seqs_a; job.sb = seqs_b; job.oa = offs_a; job.ob = offs_b; job.n_pairs = n_pairs;
    job.subst = subst; job.asz = asz; job.mode = mode; job.alpha = alpha; job.beta = beta;
    job.ops = (uint8_t *)ops; job.span = (int32_t *)span; job.out = out; job.traceback = 0;
    run_aln(&job, nthreads);
}
