/*
 * oracle_driver.c -- runs the C oracles (X-drop extension, pair split,
 * batch, substitution-table form, seed choice) on seeded random and edge-case
 * inputs.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: any out-of-bounds access, leak, signed overflow
 * or other undefined behaviour aborts the run.  Prints "ok <checks>" on
 * success; every result is also checked against the bounds it must satisfy.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "xdrop_oracle.h"

typedef struct {
    int64_t a_seed, b_seed, bin_matches, matches, found, status;
} os_seed;
int os_find_seed(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, int64_t k,
                 int64_t width, os_seed *out);

static uint64_t rng_state = 0x2002052000ull;
static uint64_t next_u64(void) {   /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)

int main(void) {
    long checks = 0;
    for (int t = 0; t < 3000; ++t) {
        const int64_t m = uniform(0, t < 2000 ? 40 : 600), n = uniform(0, t < 2000 ? 40 : 600);
        const int alph = (int)uniform(1, 4);
        uint8_t *a = malloc((size_t)m + 1), *b = malloc((size_t)n + 1);
        for (int64_t i = 0; i < m; ++i) a[i] = (uint8_t)uniform(0, alph - 1);
        for (int64_t i = 0; i < n; ++i) b[i] = (uint8_t)(t % 3 == 0 && i < m ? a[i] : uniform(0, alph - 1));
        const int64_t match = uniform(1, 4), mismatch = uniform(-4, 0), gap = uniform(-4, -1);
        const int64_t x = t % 7 == 0 ? (1 << 29) : uniform(0, 60);
        ox_ext e;
        const int64_t cap = m + n + 1;
        int64_t *buf = malloc(sizeof(int64_t) * 6 * (size_t)cap);
        ox_trace tr = {cap, 0, buf, buf + cap, buf + 2 * cap, buf + 3 * cap, buf + 4 * cap, buf + 5 * cap};
        CHECK(ox_extend(a, m, b, n, match, mismatch, gap, x, &e, &tr) == 0);
        CHECK(e.best >= 0 && e.bi >= 0 && e.bi <= m && e.bj >= 0 && e.bj <= n);
        CHECK(e.cells >= 0 && e.cells <= (m + 1) * (n + 1) - 1 + (m + n == 0));
        CHECK(tr.n <= cap);
        int64_t table[16];
        for (int q = 0; q < 16; ++q) table[q] = uniform(-5, 5);
        CHECK(ox_extend_matrix(a, m, b, n, table, gap, x, &e, NULL) == 0);
        CHECK(e.bi <= m && e.bj <= n);
        const int64_t k = uniform(0, 8);
        if (m >= k && n >= k) {
            ox_pair_result pr;
            const int64_t pa = uniform(0, m - k), pb = uniform(0, n - k);
            CHECK(ox_pair(a, m, b, n, pa, pb, k, match, mismatch, gap, x, &pr) == 0);
            CHECK(pr.status == 0 && pr.a_begin >= 0 && pr.a_end <= m && pr.b_end <= n);
            CHECK(ox_pair_matrix(a, m, b, n, pa, pb, k, table, gap, x, &pr) == 0);
            ox_pair_result bad;
            ox_pair(a, m, b, n, m, pb, k + 1, match, mismatch, gap, x, &bad);   /* seed past A */
            CHECK(bad.status == 1);
            int64_t off0 = 0, la = m, lb = n, sa = pa, sb = pb;
            int32_t xx = (int32_t)(x > (1 << 29) ? (1 << 29) : x);
            ox_batch(a, b, &off0, &la, &off0, &lb, &sa, &sb, &xx, 1, k, match, mismatch, gap, &pr);
            ox_batch_matrix(a, b, &off0, &la, &off0, &lb, &sa, &sb, &xx, 1, k, table, gap, &pr);
        }
        os_seed s;
        const int64_t sk = uniform(0, 33), width = uniform(0, 20);
        os_find_seed(a, m, b, n, sk, width, &s);
        CHECK(s.status == ((sk < 1 || sk > 31 || width < 1) ? 1 : 0));
        if (s.found) CHECK(s.a_seed + sk <= m && s.b_seed + sk <= n && memcmp(a + s.a_seed, b + s.b_seed, (size_t)sk) == 0);
        free(a);
        free(b);
        free(buf);
        checks += 1;
    }
    printf("ok %ld\n", checks);
    return 0;
}
