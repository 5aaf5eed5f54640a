/*
 * xdrop_oracle.h -- CPU reference of X-drop seed extension.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the HIP library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg call it;
 * the product path never links, loads or calls it, and it shares no code,
 * header, table or helper with the HIP library.
 *
 * Sequences are arrays of base codes 0..3 (one byte per base), 0-based in
 * memory: a[0] is the paper's a_1.
 */
#ifndef XDROP_ORACLE_H
#define XDROP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result of one one-directional extension (Section III-A, Algorithm 1). */
typedef struct {
    int64_t best;   /* best score, >= 0 (the empty extension scores 0)          */
    int64_t bi;     /* characters of A consumed at the best cell                */
    int64_t bj;     /* characters of B consumed at the best cell                */
    int64_t cells;  /* cells computed: sum over anti-diagonals of the range size */
    int64_t ndiag;  /* anti-diagonals whose range was computed                  */
    int64_t wmax;   /* widest computed range                                    */
} ox_ext;

/* Optional per-anti-diagonal trace (debugging and invariant tests). */
typedef struct {
    int64_t cap;      /* entries available in each array                        */
    int64_t n;        /* entries written (anti-diagonals 1..n)                  */
    int64_t *lo, *hi; /* computed range, i-coordinates                          */
    int64_t *la, *lb; /* live range after pruning (la > lb when empty)          */
    int64_t *best;    /* best after this anti-diagonal                          */
    int64_t *vmax;    /* max over this anti-diagonal (OX_NEG when all pruned)   */
} ox_trace;

/* Per-pair result (seed split of Section IV-B). */
typedef struct {
    int64_t score, left_score, right_score, seed_score;
    int64_t a_begin, a_end, b_begin, b_end; /* half-open, read-local             */
    int64_t left_cells, right_cells;
    int64_t left_bi, left_bj, right_bi, right_bj;
    int64_t status; /* 0 ok, 1 invalid pair (seed outside a read, k < 0, X < 0) */
} ox_pair_result;

/* -inf: a flag value, never used in arithmetic. */
#define OX_NEG INT64_MIN

/* One extension of a[0..m) against b[0..n) under a substitution table:
 * aligning base p of A with base q of B scores score[4 * p + q] (Section
 * III-A with the match/mismatch choice generalised to a table, as Section
 * VIII proposes for other alphabets).  Returns 0, or 1 on bad arguments. */
int ox_extend_matrix(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                     const int64_t score[16], int64_t gap, int64_t x,
                     ox_ext *out, ox_trace *trace);

/* Match/mismatch scoring: the table with `match` on its diagonal. */
int ox_extend(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
              int64_t match, int64_t mismatch, int64_t gap, int64_t x,
              ox_ext *out, ox_trace *trace);

/* Left and right extension of one seeded pair, combined (seed score summed
 * from the table). */
int ox_pair_matrix(const uint8_t *a, int64_t len_a, const uint8_t *b, int64_t len_b,
                   int64_t a_seed, int64_t b_seed, int64_t k,
                   const int64_t score[16], int64_t gap, int64_t x,
                   ox_pair_result *out);

/* Left and right extension of one seeded pair, combined. */
int ox_pair(const uint8_t *a, int64_t len_a, const uint8_t *b, int64_t len_b,
            int64_t a_seed, int64_t b_seed, int64_t k,
            int64_t match, int64_t mismatch, int64_t gap, int64_t x,
            ox_pair_result *out);

/* A batch laid out as arenas (see the generator).  Returns elapsed seconds
 * of the extension loop (monotonic clock), excluding nothing else. */
double ox_batch(const uint8_t *arena_a, const uint8_t *arena_b,
                const int64_t *a_off, const int64_t *a_len,
                const int64_t *b_off, const int64_t *b_len,
                const int64_t *a_seed, const int64_t *b_seed, const int32_t *x,
                int64_t n_pairs, int64_t k, int64_t match, int64_t mismatch,
                int64_t gap, ox_pair_result *out);

double ox_batch_matrix(const uint8_t *arena_a, const uint8_t *arena_b,
                       const int64_t *a_off, const int64_t *a_len,
                       const int64_t *b_off, const int64_t *b_len,
                       const int64_t *a_seed, const int64_t *b_seed, const int32_t *x,
                       int64_t n_pairs, int64_t k, const int64_t score[16], int64_t gap,
                       ox_pair_result *out);

#ifdef __cplusplus
}
#endif
#endif
