/*
 * seed_oracle.c -- plain CPU reference of the seed choice that feeds the
 * X-drop extension: one exact shared k-mer per read pair.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite calls it; the product path
 * never links, loads or calls it, and it shares no code with the HIP library.
 *
 * The paper's application (Section V) picks the k-mer that starts each
 * extension by binning: the positions of the k-mers two reads share estimate
 * their overlap, the shared k-mers are binned by it and the consensus bin
 * supplies the seed.  The paper gives no formula, so this is the reading:
 *   - matches: every (p, q) with A[p, p+k) == B[q, q+k) exactly;
 *   - a match lies on diagonal q - p; diagonals are binned in bands of
 *     `width`, bin floor((q - p) / width);
 *   - the bin holding the most matches wins, ties going to the lower bin;
 *   - the seed is the winning bin's match with the smallest p, then the
 *     smallest q.
 * Reads without a shared k-mer have no seed.  The k-mers of B are sorted with
 * their positions and each k-mer of A is looked up by binary search: slow and
 * plain, one pair at a time.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t a_seed, b_seed;  /* the chosen match (0, 0 when none)           */
    int64_t bin_matches;     /* matches in the winning bin                  */
    int64_t matches;         /* all matches                                 */
    int64_t found;           /* 1 when the reads share a k-mer              */
    int64_t status;          /* 0 ok, 1 bad arguments                       */
} os_seed;

typedef struct {
    uint64_t code;
    int64_t pos;
} kmer_at;

/* The k bases from s[0] as one number, base t in bits 2(k-1-t), 2(k-1-t)+1. */
static uint64_t kmer_code(const uint8_t *s, int64_t k) {
    uint64_t c = 0;
    for (int64_t t = 0; t < k; t++) c = (c << 2) | (uint64_t)(s[t] & 3);
    return c;
}

static int by_code_then_pos(const void *x, const void *y) {
    const kmer_at *u = (const kmer_at *)x, *v = (const kmer_at *)y;
    if (u->code != v->code) return u->code < v->code ? -1 : 1;
    if (u->pos != v->pos) return u->pos < v->pos ? -1 : 1;
    return 0;
}

/* floor(num / den) for den > 0 */
static int64_t floor_div(int64_t num, int64_t den) {
    int64_t q = num / den;
    if ((num % den != 0) && (num < 0)) q -= 1;
    return q;
}

int os_find_seed(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, int64_t k,
                 int64_t width, os_seed *out) {
    memset(out, 0, sizeof(*out));
    if (k < 1 || k > 31 || width < 1 || m < 0 || n < 0) {
        out->status = 1;
        return 1;
    }
    if (m < k || n < k) return 0;
    const int64_t nb = n - k + 1;
    kmer_at *tab = (kmer_at *)malloc(sizeof(kmer_at) * (size_t)nb);
    for (int64_t q = 0; q < nb; q++) {
        tab[q].code = kmer_code(b + q, k);
        tab[q].pos = q;
    }
    qsort(tab, (size_t)nb, sizeof(kmer_at), by_code_then_pos);

    const int64_t lo_bin = floor_div(-(m - k), width);
    const int64_t hi_bin = floor_div(n - k, width);
    const int64_t nbins = hi_bin - lo_bin + 1;
    int64_t *count = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
    int64_t *fp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbins);
    int64_t *fq = (int64_t *)malloc(sizeof(int64_t) * (size_t)nbins);
    for (int64_t i = 0; i < nbins; i++) fp[i] = fq[i] = -1;

    for (int64_t p = 0; p + k <= m; p++) {
        const uint64_t c = kmer_code(a + p, k);
        int64_t lo = 0, hi = nb;                 /* first entry with code >= c */
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (tab[mid].code < c) lo = mid + 1;
            else hi = mid;
        }
        for (int64_t e = lo; e < nb && tab[e].code == c; e++) {
            const int64_t q = tab[e].pos;
            const int64_t bin = floor_div(q - p, width) - lo_bin;
            count[bin] += 1;
            out->matches += 1;
            if (fp[bin] < 0 || p < fp[bin] || (p == fp[bin] && q < fq[bin])) {
                fp[bin] = p;
                fq[bin] = q;
            }
        }
    }
    if (out->matches > 0) {
        int64_t win = 0;
        for (int64_t i = 1; i < nbins; i++)
            if (count[i] > count[win]) win = i;   /* strict: the lower bin keeps a tie */
        out->found = 1;
        out->a_seed = fp[win];
        out->b_seed = fq[win];
        out->bin_matches = count[win];
    }
    free(tab);
    free(count);
    free(fp);
    free(fq);
    return 0;
}

/* Every pair of a batch laid out as arenas of base codes. */
void os_find_seeds(const uint8_t *arena_a, const uint8_t *arena_b, const int64_t *a_off,
                   const int64_t *a_len, const int64_t *b_off, const int64_t *b_len,
                   int64_t n_pairs, int64_t k, int64_t width, os_seed *out) {
    for (int64_t p = 0; p < n_pairs; p++)
        os_find_seed(arena_a + a_off[p], a_len[p], arena_b + b_off[p], b_len[p], k, width,
                     &out[p]);
}
