/*
 * Driver for the sanitizer build of the C oracle (test infrastructure: built and run by
 * the CPU test suite with AddressSanitizer and UndefinedBehaviorSanitizer).  It calls
 * every routine of csk_oracle.c on small seeded inputs, edge cases included (no tuples,
 * one bucket, counters that wrap), and checks linearity: the sketch of a stream equals
 * the sum of the sketches of its halves.  Exit status 0 when every check holds.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t or_poly_hash(const uint64_t *coef, int deg, uint32_t x);
int or_sign(const uint64_t *coef4, uint32_t x);
uint64_t or_bin(const uint64_t *coef2, uint32_t x, uint64_t m);
void or_create_sketch(int32_t n_cols, const int32_t *col_comp, const int32_t *col_nedges,
                      const int32_t *col_edges, int32_t max_edges, int32_t d, uint64_t m,
                      const uint64_t *sign_coef, int32_t n_edges, const uint64_t *bin_coef, int32_t n_comps,
                      const uint32_t *keys, const int64_t *weights, uint64_t n, int64_t *sketch);
void or_create_ams_sketch(int32_t n_cols, const int32_t *col_nedges, const int32_t *col_edges,
                          int32_t max_edges, int32_t d, uint64_t m, const uint64_t *ams_coef,
                          int32_t n_edges, const uint32_t *keys, const int64_t *weights, uint64_t n,
                          int64_t *sketch);
void or_accumulate(const uint64_t *bins, const int32_t *signs, const int64_t *weights, uint64_t n, uint64_t m,
                   int64_t *sketch);

static uint64_t state = 12345;
static uint64_t next(void)
{
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main(void)
{
    enum { D = 3, E = 3, Q = 2, N = 257, COLS = 2, MAXE = 2 };
    uint64_t sign[D * E * 4], bin[D * Q * 2], ams[D * 5 * E * 4];
    for (size_t i = 0; i < sizeof(sign) / 8; ++i) sign[i] = next() >> 3;
    for (size_t i = 0; i < sizeof(bin) / 8; ++i) bin[i] = next() >> 3;
    for (size_t i = 0; i < sizeof(ams) / 8; ++i) ams[i] = next() >> 3;
    /* a relation with two key columns: column 0 in two joins, column 1 in one */
    const int32_t comp[COLS] = {0, 1}, nedges[COLS] = {2, 1}, edges[COLS * MAXE] = {0, 1, 2, 0};
    uint32_t keys[N * COLS];
    int64_t w[N];
    for (int i = 0; i < N * COLS; ++i) keys[i] = (uint32_t)next();
    for (int i = 0; i < N; ++i) w[i] = (int64_t)(next() >> 1) - (int64_t)(1ull << 62); /* wraps */
    const uint64_t ms[] = {1, 2, 7, 64};
    for (int mi = 0; mi < 4; ++mi) {
        const uint64_t m = ms[mi];
        int64_t *all = calloc(D * m, 8), *half = calloc(D * m, 8), *zero = calloc(D * m, 8);
        or_create_sketch(COLS, comp, nedges, edges, MAXE, D, m, sign, E, bin, Q, keys, w, N, all);
        or_create_sketch(COLS, comp, nedges, edges, MAXE, D, m, sign, E, bin, Q, keys, w, 100, half);
        or_create_sketch(COLS, comp, nedges, edges, MAXE, D, m, sign, E, bin, Q, keys + 100 * COLS, w + 100,
                         N - 100, half);
        CHECK(memcmp(all, half, D * m * 8) == 0);
        or_create_sketch(COLS, comp, nedges, edges, MAXE, D, m, sign, E, bin, Q, keys, NULL, 0, zero);
        for (uint64_t j = 0; j < D * m; ++j) CHECK(zero[j] == 0);
        free(all);
        free(half);
        free(zero);
    }
    {
        const uint64_t m = 5;
        int64_t all[D * 5] = {0}, half[D * 5] = {0};
        or_create_ams_sketch(COLS, nedges, edges, MAXE, D, m, ams, E, keys, w, N, all);
        or_create_ams_sketch(COLS, nedges, edges, MAXE, D, m, ams, E, keys, w, 100, half);
        or_create_ams_sketch(COLS, nedges, edges, MAXE, D, m, ams, E, keys + 100 * COLS, w + 100, N - 100, half);
        CHECK(memcmp(all, half, sizeof(all)) == 0);
    }
    {
        uint64_t bins[N];
        int32_t signs[N];
        int64_t c[16] = {0};
        for (int i = 0; i < N; ++i) {
            bins[i] = next();
            signs[i] = (next() & 1) ? 1 : -1;
        }
        or_accumulate(bins, signs, w, N, 16, c);
        int64_t ref[16] = {0};
        for (int i = 0; i < N; ++i)
            ref[bins[i] % 16] = (int64_t)((uint64_t)ref[bins[i] % 16] + (uint64_t)(int64_t)signs[i] * (uint64_t)w[i]);
        CHECK(memcmp(c, ref, sizeof(c)) == 0);
    }
    CHECK(or_poly_hash(sign, 3, 0) == sign[0] % ((1ull << 61) - 1));
    CHECK(or_bin(bin, 0xFFFFFFFFu, 1) == 0);
    CHECK(or_sign(sign, 7) == 1 || or_sign(sign, 7) == -1);
    if (fails) return 1;
    printf("sanitize driver: all checks passed\n");
    return 0;
}
