/*
 * ga_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU oracle for the guided extension
 * alignment of AGAThA (PPoPP'24, arXiv 2403.06478). Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load this file's
 * library; the product path never does. It shares no code, header or table
 * with the HIP implementation.
 *
 * What it computes (Section 2.1, Eq. 1-3 for the score table, Eq. 4-7 for the
 * termination condition). Where the paper is silent the following readings
 * are taken: gap runs are charged per maximal run; the z-drop slope beta is
 * the long-piece extension e2; i' < i and j' < j are strict; every non-empty
 * anti-diagonal is tested; ties inside an anti-diagonal go to the smallest i
 * and the global maximum moves only on a strictly larger value; only interior
 * cells enter the maxima; w < 0 disables the band and Z < 0 the z-drop.
 *
 *   S(x,y)  = -ambig if x or y is N, +a if x == y, -b otherwise.
 *   gamma(l)= min(q + l*e, q2 + l*e2)   (two-piece affine gap of length l;
 *             Eq. 2-3 are the one-piece case alpha = q+e, beta = e).
 *   Band:   lattice point (i,j) is usable iff w < 0 or |i-j| <= w, including
 *           the boundary points with i = -1 or j = -1.
 *   For in-band 0 <= i < n, 0 <= j < m and k = 1,2:
 *     E_k(i,j) = max(H(i-1,j) - (q_k+e_k), E_k(i-1,j) - e_k)   (consumes T[i])
 *     F_k(i,j) = max(H(i,j-1) - (q_k+e_k), F_k(i,j-1) - e_k)   (consumes Q[j])
 *     H(i,j)   = max(H(i-1,j-1) + S(T[i],Q[j]), E_1, E_2, F_1, F_2)
 *   Boundary: H(-1,-1) = 0, H(i,-1) = -gamma(i+1), H(-1,j) = -gamma(j+1);
 *             E_k(-1,.) = F_k(.,-1) = -inf; out-of-band points are -inf.
 *
 *   Sweep (Eq. 4-7): G = 0 at (-1,-1). For anti-diagonals r = i+j = 0..n+m-2
 *   with at least one in-band cell: M = max H on r, (mi,mj) the cell with the
 *   smallest i attaining it; end := (M,mi,mj). If M > G the global maximum
 *   moves there; otherwise, if Z >= 0, mi > gi, mj > gj and
 *   G - M > Z + e2*|(mi-gi) - (mj-gj)|, the alignment is z-dropped and the
 *   sweep stops.
 *
 * Arithmetic is int64 so no input inside the library's range guard can
 * overflow here. Storage is three anti-diagonals indexed by i.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t a, b, q, e, q2, e2, ambig; } orc_scoring_t;
typedef struct {
    int32_t max_score, max_i, max_j, end_score, end_i, end_j, zdropped;
} orc_result_t;

#define NEG_INF (INT64_MIN / 4)

typedef struct { int64_t H, E1, E2, F1, F2; } cell_t;

static int base_code(uint8_t c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4; /* N: anything outside ACGT */
    }
}

/* Substitution score S (Section 2.1). */
static int64_t subst(const orc_scoring_t *sc, uint8_t x, uint8_t y) {
    int cx = base_code(x), cy = base_code(y);
    if (cx == 4 || cy == 4) return -(int64_t)sc->ambig;
    return cx == cy ? (int64_t)sc->a : -(int64_t)sc->b;
}

/* Cost of one gap run of length l >= 1 (Eq. 2-3 generalised to two pieces). */
static int64_t gap_cost(const orc_scoring_t *sc, int64_t l) {
    int64_t c1 = (int64_t)sc->q + l * sc->e;
    int64_t c2 = (int64_t)sc->q2 + l * sc->e2;
    return c1 < c2 ? c1 : c2;
}

static int in_band(int64_t i, int64_t j, int32_t w) {
    if (w < 0) return 1;
    int64_t d = i - j;
    if (d < 0) d = -d;
    return d <= w;
}

static int64_t max2(int64_t x, int64_t y) { return x > y ? x : y; }

static cell_t neg_cell(void) {
    cell_t c = {NEG_INF, NEG_INF, NEG_INF, NEG_INF, NEG_INF};
    return c;
}

/* State of lattice point (i,j), i,j >= -1, taken from the anti-diagonal array
 * that holds anti-diagonal i+j (interior points) or from the boundary. */
static cell_t get_cell(const orc_scoring_t *sc, int32_t w, const cell_t *diag_arr,
                       int64_t i, int64_t j) {
    if (!in_band(i, j, w)) return neg_cell();
    cell_t c = neg_cell();
    if (i < 0 && j < 0) { c.H = 0; return c; }
    if (i < 0) { c.H = -gap_cost(sc, j + 1); return c; }
    if (j < 0) { c.H = -gap_cost(sc, i + 1); return c; }
    return diag_arr[i];
}

/* Range of interior in-band rows on anti-diagonal r; returns 0 if empty. */
static int diag_range(int64_t n, int64_t m, int32_t w, int64_t r, int64_t *lo, int64_t *hi) {
    int64_t l = r - (m - 1);
    if (l < 0) l = 0;
    int64_t h = r < n - 1 ? r : n - 1;
    if (w >= 0) {
        /* |i - (r-i)| <= w  <=>  (r-w)/2 <= i <= (r+w)/2 */
        int64_t t = r - w;
        int64_t lb = t >= 0 ? (t + 1) / 2 : -((-t) / 2); /* ceil(t/2) */
        int64_t u = r + w;
        int64_t ub = u >= 0 ? u / 2 : -((-u + 1) / 2);   /* floor(u/2) */
        if (lb > l) l = lb;
        if (ub < h) h = ub;
    }
    *lo = l;
    *hi = h;
    return l <= h;
}

int oracle_align(const uint8_t *T, int32_t n, const uint8_t *Q, int32_t m,
                 const orc_scoring_t *sc, int32_t w, int32_t Z,
                 orc_result_t *out, int64_t *cells_out) {
    orc_result_t res = {0, -1, -1, 0, -1, -1, 0};
    int64_t cells = 0;
    if (n <= 0 || m <= 0) {
        *out = res;
        if (cells_out) *cells_out = 0;
        return 0;
    }
    cell_t *arr[3];
    for (int k = 0; k < 3; ++k) {
        arr[k] = (cell_t *)malloc(sizeof(cell_t) * (size_t)n);
        if (!arr[k]) { for (int t = 0; t < k; ++t) free(arr[t]); return -1; }
    }
    int64_t G = 0, gi = -1, gj = -1;
    for (int64_t r = 0; r <= (int64_t)n + m - 2; ++r) {
        cell_t *cur = arr[r % 3];
        const cell_t *prev = arr[(r + 2) % 3];  /* anti-diagonal r-1 */
        const cell_t *prev2 = arr[(r + 1) % 3]; /* anti-diagonal r-2 */
        int64_t lo, hi;
        if (!diag_range(n, m, w, r, &lo, &hi)) continue;
        int64_t M = 0, mi = -1, mj = -1;
        int have = 0;
        for (int64_t i = lo; i <= hi; ++i) {
            int64_t j = r - i;
            cell_t up = get_cell(sc, w, prev, i - 1, j);
            cell_t left = get_cell(sc, w, prev, i, j - 1);
            cell_t dg = get_cell(sc, w, prev2, i - 1, j - 1);
            cell_t c;
            c.E1 = max2(up.H - ((int64_t)sc->q + sc->e), up.E1 - sc->e);
            c.E2 = max2(up.H - ((int64_t)sc->q2 + sc->e2), up.E2 - sc->e2);
            c.F1 = max2(left.H - ((int64_t)sc->q + sc->e), left.F1 - sc->e);
            c.F2 = max2(left.H - ((int64_t)sc->q2 + sc->e2), left.F2 - sc->e2);
            int64_t h = dg.H + subst(sc, T[i], Q[j]);
            h = max2(h, c.E1);
            h = max2(h, c.E2);
            h = max2(h, c.F1);
            h = max2(h, c.F2);
            c.H = h;
            cur[i] = c;
            if (!have || h > M) { M = h; mi = i; mj = j; have = 1; } /* smallest i on ties */
        }
        cells += hi - lo + 1;
        res.end_score = (int32_t)M;
        res.end_i = (int32_t)mi;
        res.end_j = (int32_t)mj;
        if (M > G) {
            G = M; gi = mi; gj = mj;
        } else if (Z >= 0 && mi > gi && mj > gj) {
            int64_t dd = (mi - gi) - (mj - gj);
            if (dd < 0) dd = -dd;
            if (G - M > (int64_t)Z + (int64_t)sc->e2 * dd) {
                res.zdropped = 1;
                break;
            }
        }
    }
    res.max_score = (int32_t)G;
    res.max_i = (int32_t)gi;
    res.max_j = (int32_t)gj;
    for (int k = 0; k < 3; ++k) free(arr[k]);
    *out = res;
    if (cells_out) *cells_out = cells;
    return 0;
}

/* ---- many pairs: one pair per worker thread, pulled from an atomic counter */

typedef struct {
    int64_t n_pairs;
    const uint8_t *tseq; const int64_t *toff; const int32_t *tlen;
    const uint8_t *qseq; const int64_t *qoff; const int32_t *qlen;
    const orc_scoring_t *sc; int32_t w, Z;
    orc_result_t *out; int64_t *cells;
    atomic_llong next;
    atomic_int err;
} batch_job_t;

static void *batch_worker(void *arg) {
    batch_job_t *job = (batch_job_t *)arg;
    for (;;) {
        int64_t p = atomic_fetch_add(&job->next, 1);
        if (p >= job->n_pairs) break;
        int64_t c = 0;
        if (oracle_align(job->tseq + job->toff[p], job->tlen[p], job->qseq + job->qoff[p],
                         job->qlen[p], job->sc, job->w, job->Z, &job->out[p], &c) != 0)
            atomic_store(&job->err, 1);
        if (job->cells) job->cells[p] = c;
    }
    return NULL;
}

int oracle_align_batch(int64_t n_pairs, const uint8_t *tseq, const int64_t *toff,
                       const int32_t *tlen, const uint8_t *qseq, const int64_t *qoff,
                       const int32_t *qlen, const orc_scoring_t *sc, int32_t w, int32_t Z,
                       orc_result_t *out, int64_t *cells, int32_t nthreads) {
    batch_job_t job;
    job.n_pairs = n_pairs; job.tseq = tseq; job.toff = toff; job.tlen = tlen;
    job.qseq = qseq; job.qoff = qoff; job.qlen = qlen; job.sc = sc; job.w = w; job.Z = Z;
    job.out = out; job.cells = cells;
    atomic_init(&job.next, 0);
    atomic_init(&job.err, 0);
    if (nthreads < 1) nthreads = 1;
    if (nthreads == 1) {
        batch_worker(&job);
    } else {
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
        if (!th) return -1;
        int started = 0;
        for (int t = 0; t < nthreads; ++t)
            if (pthread_create(&th[t], NULL, batch_worker, &job) == 0) ++started;
        if (started == 0) batch_worker(&job);
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
    }
    return atomic_load(&job.err) ? -1 : 0;
}
