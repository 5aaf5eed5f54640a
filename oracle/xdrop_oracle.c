/*
 * xdrop_oracle.c -- plain, slow, single-threaded CPU reference of X-drop seed
 * extension (LOGAN, arXiv 2002.05200).
 *
 * TEST INFRASTRUCTURE ONLY: see xdrop_oracle.h.
 *
 * X-drop is a heuristic, so this oracle is the algorithm itself, step by step,
 * in the paper's order:
 *   - problem statement and cell recurrence (Section III-A): S(i,j) takes the
 *     best of the diagonal predecessor plus the substitution score of
 *     (a_i, b_j) and the two neighbours plus the (negative) gap score; the
 *     paper's match/mismatch choice is the table with `match` on its
 *     diagonal, and any 4 x 4 table is accepted (Section VIII names other
 *     scoring schemes as future work);
 *   - X-drop rule (Section III-A): a cell scoring below best - X becomes -inf
 *     and is never used again; best is updated once per anti-diagonal, after
 *     the whole anti-diagonal is computed (Section IV-A);
 *   - Algorithm 1: three rolling anti-diagonals, running best, trimming of the
 *     -inf runs at both ends, loop until the anti-diagonal is empty;
 *   - Algorithm 2: every cell of the anti-diagonal computed independently;
 *   - seed split (Section IV-B): a pair becomes a left extension on the
 *     reversed prefixes and a right extension on the suffixes.
 * The readings taken where the paper is garbled or silent are:
 *   - max over the applicable predecessors; signed additive scores;
 *   - prune iff value < best - X (strict), with best as of the end of the
 *     previous anti-diagonal; best never decreases;
 *   - only the leading and trailing -inf runs are trimmed; the next range is
 *     [first live, last live + 1] clipped to the (m+1) x (n+1) matrix;
 *   - stop when the live range is empty or d = m + n;
 *   - the reported end is the best cell: first anti-diagonal reaching the
 *     final best, smallest i on it;
 *   - both directions start at best = 0 and ignore the seed and each other;
 *   - cells = sum over anti-diagonals of the computed range size.
 * Scores are int64 and -inf is a flag value that never enters arithmetic,
 * so the result is exact for any X.
 */
#define _POSIX_C_SOURCE 199309L
#include "xdrop_oracle.h"

#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef struct {
    int64_t lo, hi;  /* i-range stored (lo > hi: empty)          */
    int64_t *v;      /* v[i - lo] for lo <= i <= hi              */
} antidiag;

/* Value of cell i of an anti-diagonal; -inf outside its computed range. */
static int64_t cell(const antidiag *ad, int64_t i) {
    if (i < ad->lo || i > ad->hi) return OX_NEG;
    return ad->v[i - ad->lo];
}

static int64_t max2(int64_t p, int64_t q) { return p > q ? p : q; }
static int64_t min2(int64_t p, int64_t q) { return p < q ? p : q; }

int ox_extend_matrix(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                     const int64_t score[16], int64_t gap, int64_t x,
                     ox_ext *out, ox_trace *trace) {
    if (m < 0 || n < 0 || x < 0 || x > (INT64_C(1) << 62) || !out) return 1;
    memset(out, 0, sizeof(*out));
    if (trace) trace->n = 0;

    int64_t cap = min2(m, n) + 2;
    antidiag ad[3];
    for (int t = 0; t < 3; t++) {
        ad[t].v = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        if (!ad[t].v) {
            for (int u = 0; u < t; u++) free(ad[u].v);
            return 1;
        }
    }
    /* d - 2, d - 1, d: rotated after every anti-diagonal. */
    antidiag *two_back = &ad[0], *one_back = &ad[1], *cur = &ad[2];

    /* Anti-diagonal 0 is the origin cell, score 0. */
    two_back->lo = 1; two_back->hi = 0;          /* empty */
    one_back->lo = 0; one_back->hi = 0; one_back->v[0] = 0;
    int64_t live_lo = 0, live_hi = 0;
    int64_t best = 0, bi = 0, bj = 0, cells = 0, ndiag = 0, wmax = 0;

    for (int64_t d = 1; d <= m + n; d++) {
        /* Range of this anti-diagonal from the trimmed previous one. */
        int64_t lo = max2(live_lo, d - n);
        int64_t hi = min2(live_hi + 1, m);
        if (lo > hi) break;

        int64_t threshold = best - x;   /* best as of the end of d - 1 */
        cur->lo = lo; cur->hi = hi;
        for (int64_t i = lo; i <= hi; i++) {
            int64_t j = d - i;
            /* Best over the predecessors that exist and are not -inf. */
            int64_t v = OX_NEG, p;
            if (i >= 1 && j >= 1) {                     /* (i-1, j-1) */
                p = cell(two_back, i - 1);
                if (p != OX_NEG) {
                    int64_t s = score[4 * a[i - 1] + b[j - 1]];
                    v = max2(v, p + s);
                }
            }
            if (i >= 1) {                               /* (i-1, j)   */
                p = cell(one_back, i - 1);
                if (p != OX_NEG) v = max2(v, p + gap);
            }
            if (j >= 1) {                               /* (i, j-1)   */
                p = cell(one_back, i);
                if (p != OX_NEG) v = max2(v, p + gap);
            }
            /* X-drop: below best - X becomes -inf for good. */
            cur->v[i - lo] = (v == OX_NEG || v < threshold) ? OX_NEG : v;
        }
        cells += hi - lo + 1;
        ndiag += 1;
        if (hi - lo + 1 > wmax) wmax = hi - lo + 1;

        /* Trim: first and last surviving cell. */
        int64_t first = -1, last = -1, vmax = OX_NEG, imax = -1;
        for (int64_t i = lo; i <= hi; i++) {
            int64_t v = cur->v[i - lo];
            if (v == OX_NEG) continue;
            if (first < 0) first = i;
            last = i;
            if (v > vmax) { vmax = v; imax = i; }   /* strict: smallest i wins */
        }
        if (first >= 0 && vmax > best) {
            best = vmax; bi = imax; bj = d - imax;
        }
        if (trace && trace->n < trace->cap) {
            int64_t e = trace->n++;
            trace->lo[e] = lo; trace->hi[e] = hi;
            trace->la[e] = first >= 0 ? first : 1;
            trace->lb[e] = first >= 0 ? last : 0;
            trace->best[e] = best; trace->vmax[e] = vmax;
        }
        if (first < 0) break;
        live_lo = first; live_hi = last;

        antidiag *t = two_back; two_back = one_back; one_back = cur; cur = t;
    }

    out->best = best; out->bi = bi; out->bj = bj;
    out->cells = cells; out->ndiag = ndiag; out->wmax = wmax;
    for (int t = 0; t < 3; t++) free(ad[t].v);
    return 0;
}

/* Match/mismatch scoring is the substitution table with `match` on its
 * diagonal and `mismatch` everywhere else. */
static void linear_table(int64_t match, int64_t mismatch, int64_t score[16]) {
    for (int p = 0; p < 4; p++)
        for (int q = 0; q < 4; q++) score[4 * p + q] = (p == q) ? match : mismatch;
}

int ox_extend(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int64_t match, int64_t mismatch, int64_t gap, int64_t x,
              ox_ext *out, ox_trace *trace) {
    int64_t score[16];
    linear_table(match, mismatch, score);
    return ox_extend_matrix(a, m, b, n, score, gap, x, out, trace);
}

int ox_pair_matrix(const uint8_t *a, int64_t len_a, const uint8_t *b, int64_t len_b,
                   int64_t a_seed, int64_t b_seed, int64_t k,
                   const int64_t score[16], int64_t gap, int64_t x,
                   ox_pair_result *out) {
    memset(out, 0, sizeof(*out));
    if (k < 0 || x < 0 || a_seed < 0 || b_seed < 0 || a_seed + k > len_a ||
        b_seed + k > len_b) {
        out->status = 1;
        return 1;
    }
    /* Right extension: the suffixes after the seed, read forward. */
    ox_ext right, left;
    int rc = ox_extend_matrix(a + a_seed + k, len_a - a_seed - k, b + b_seed + k,
                              len_b - b_seed - k, score, gap, x, &right, NULL);
    /* Left extension: the prefixes before the seed, reversed. */
    uint8_t *ra = (uint8_t *)malloc((size_t)(a_seed > 0 ? a_seed : 1));
    uint8_t *rb = (uint8_t *)malloc((size_t)(b_seed > 0 ? b_seed : 1));
    for (int64_t t = 0; t < a_seed; t++) ra[t] = a[a_seed - 1 - t];
    for (int64_t t = 0; t < b_seed; t++) rb[t] = b[b_seed - 1 - t];
    rc |= ox_extend_matrix(ra, a_seed, rb, b_seed, score, gap, x, &left, NULL);
    free(ra); free(rb);
    if (rc) { out->status = 1; return 1; }

    int64_t seed_score = 0;
    for (int64_t t = 0; t < k; t++)
        seed_score += score[4 * a[a_seed + t] + b[b_seed + t]];

    out->left_score = left.best;
    out->right_score = right.best;
    out->seed_score = seed_score;
    out->score = left.best + seed_score + right.best;
    out->a_begin = a_seed - left.bi;
    out->a_end = a_seed + k + right.bi;
    out->b_begin = b_seed - left.bj;
    out->b_end = b_seed + k + right.bj;
    out->left_cells = left.cells;
    out->right_cells = right.cells;
    out->left_bi = left.bi; out->left_bj = left.bj;
    out->right_bi = right.bi; out->right_bj = right.bj;
    out->status = 0;
    return 0;
}

int ox_pair(const uint8_t *a, int64_t len_a, const uint8_t *b, int64_t len_b,
            int64_t a_seed, int64_t b_seed, int64_t k,
            int64_t match, int64_t mismatch, int64_t gap, int64_t x,
            ox_pair_result *out) {
    int64_t score[16];
    linear_table(match, mismatch, score);
    return ox_pair_matrix(a, len_a, b, len_b, a_seed, b_seed, k, score, gap, x, out);
}

double ox_batch_matrix(const uint8_t *arena_a, const uint8_t *arena_b,
                       const int64_t *a_off, const int64_t *a_len,
                       const int64_t *b_off, const int64_t *b_len,
                       const int64_t *a_seed, const int64_t *b_seed, const int32_t *x,
                       int64_t n_pairs, int64_t k, const int64_t score[16], int64_t gap,
                       ox_pair_result *out) {
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t p = 0; p < n_pairs; p++) {
        ox_pair_matrix(arena_a + a_off[p], a_len[p], arena_b + b_off[p], b_len[p],
                       a_seed[p], b_seed[p], k, score, gap, x[p], &out[p]);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}

double ox_batch(const uint8_t *arena_a, const uint8_t *arena_b,
                const int64_t *a_off, const int64_t *a_len,
                const int64_t *b_off, const int64_t *b_len,
                const int64_t *a_seed, const int64_t *b_seed, const int32_t *x,
                int64_t n_pairs, int64_t k, int64_t match, int64_t mismatch,
                int64_t gap, ox_pair_result *out) {
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t p = 0; p < n_pairs; p++) {
        ox_pair(arena_a + a_off[p], a_len[p], arena_b + b_off[p], b_len[p],
                a_seed[p], b_seed[p], k, match, mismatch, gap, x[p], &out[p]);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
