/*
 * CPU oracle for the convolution Count sketch: the slow, plain C side.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library is
 * checked against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header or table with the GPU library.
 *
 * What is here:
 *   or_poly_hash     - a polynomial hash over the Mersenne prime field p = 2^61 - 1,
 *                      evaluated with exact 128-bit arithmetic and the C `%` operator
 *                      (Sec. 4 setup: random polynomials over a Mersenne prime field).
 *   or_create_ams_sketch - the AMS multi-join sketch of Eq. 1 (the baseline of Sec. 2):
 *                      every counter j of every repetition has its own sign polynomial
 *                      per join; a tuple adds Delta times the product of its joins'
 *                      signs to every counter.
 *   or_create_sketch - the sketch creation procedure (Alg. 2; Eq. 2-4): per tuple,
 *                      sum the bin hashes of the joined attributes modulo m, multiply
 *                      the sign hashes of every join the attribute takes part in, then
 *                      add sign * Delta to that counter.  Repeated for each of the d
 *                      independent repetitions (the l medians of Sec. 3.3), each with
 *                      its own hash coefficients.
 *
 * Conventions the paper leaves open (they are the project's reading, shared with the
 * GPU side only through this written description):
 *   - sign value  s(x) = +1 if (a0 + a1 x + a2 x^2 + a3 x^3 mod p) is even, else -1
 *   - bin value   h(x) = (b0 + b1 x mod p) mod m
 *   - counters are 64-bit two's complement and wrap on overflow.
 */
#include <stdint.h>
#include <stddef.h>

typedef unsigned __int128 u128;

static const uint64_t OR_P = (((uint64_t)1) << 61) - 1;

/* Horner evaluation of sum_i coef[i] x^i mod p, deg = number of coefficients - 1. */
uint64_t or_poly_hash(const uint64_t *coef, int deg, uint32_t x)
{
    u128 v = coef[deg] % OR_P;
    for (int i = deg - 1; i >= 0; --i)
        v = (v * (u128)x + (u128)coef[i]) % OR_P;
    return (uint64_t)v;
}

int or_sign(const uint64_t *coef4, uint32_t x)
{
    return (or_poly_hash(coef4, 3, x) & 1u) ? -1 : 1;
}

uint64_t or_bin(const uint64_t *coef2, uint32_t x, uint64_t m)
{
    return or_poly_hash(coef2, 1, x) % m;
}

/*
 * Sketch creation (Alg. 2) for one relation R_k, all d repetitions.
 *
 *   n_cols      number of joined attributes of R_k (|Omega(R_k)|), key columns in
 *               ascending attribute id
 *   col_comp    [n_cols] graph component Psi(u) of each column's attribute u
 *   col_nedges  [n_cols] number of joins at that attribute (|Gamma(u)|)
 *   col_edges   [n_cols][max_edges] edge index of each join {u, v}, v in Gamma(u)
 *   sign_coef   [d][n_edges][4]  coefficients a0..a3 of each join's sign polynomial
 *   bin_coef    [d][n_comps][2]  coefficients b0, b1 of each component's bin polynomial
 *   keys        [n][n_cols] tuple-major uint32 keys
 *   weights     [n] frequency changes Delta, or NULL for Delta = +1
 *   sketch      [d][m] int64 counters, accumulated into (not cleared)
 */
void or_create_sketch(int32_t n_cols, const int32_t *col_comp, const int32_t *col_nedges,
                      const int32_t *col_edges, int32_t max_edges,
                      int32_t d, uint64_t m,
                      const uint64_t *sign_coef, int32_t n_edges,
                      const uint64_t *bin_coef, int32_t n_comps,
                      const uint32_t *keys, const int64_t *weights, uint64_t n,
                      int64_t *sketch)
{
    for (int32_t t = 0; t < d; ++t) {
        const uint64_t *a_t = sign_coef + (size_t)t * n_edges * 4;
        const uint64_t *b_t = bin_coef + (size_t)t * n_comps * 2;
        uint64_t *c = (uint64_t *)(sketch + (size_t)t * m);
        for (uint64_t i = 0; i < n; ++i) {
            int64_t x = 1;   /* accumulated sign */
            uint64_t j = 0;  /* accumulated bin */
            for (int32_t col = 0; col < n_cols; ++col) {
                uint32_t key = keys[i * (uint64_t)n_cols + col];
                j += or_bin(b_t + 2 * col_comp[col], key, m);
                for (int32_t e = 0; e < col_nedges[col]; ++e) {
                    int32_t edge = col_edges[col * max_edges + e];
                    x = or_sign(a_t + 4 * edge, key) * x;
                }
            }
            j = j % m;
            int64_t delta = weights ? weights[i] : 1;
            /* unsigned arithmetic: the counter wraps modulo 2^64 */
            c[j] += (uint64_t)x * (uint64_t)delta;
        }
    }
}

/*
 * Sketch creation with the tuple-level hashes supplied directly, for worked examples:
 *   bins[n], signs[n] are H_k(i) and S_k(i) of each tuple, weights[n] its Delta.
 */
void or_accumulate(const uint64_t *bins, const int32_t *signs, const int64_t *weights,
                   uint64_t n, uint64_t m, int64_t *sketch)
{
    uint64_t *c = (uint64_t *)sketch;
    for (uint64_t i = 0; i < n; ++i)
        c[bins[i] % m] += (uint64_t)(int64_t)signs[i] * (uint64_t)weights[i];
}

/*
 * AMS multi-join sketch (Eq. 1) of one relation R_k, all d x m counters:
 *   c[t][j] = sum_i Delta_i * prod_{u in Omega(R_k)} prod_{v in Gamma(u)} s_{t,j,{u,v}}(i_u)
 *
 *   col_nedges  [n_cols] joins at each key column's attribute
 *   col_edges   [n_cols][max_edges] edge index of each join
 *   ams_coef    [d][m][n_edges][4]  sign polynomial a0..a3 of join e for counter j of
 *               repetition t
 *   keys, weights, n as in or_create_sketch; sketch [d][m] accumulated into.
 */
void or_create_ams_sketch(int32_t n_cols, const int32_t *col_nedges, const int32_t *col_edges,
                          int32_t max_edges, int32_t d, uint64_t m, const uint64_t *ams_coef,
                          int32_t n_edges, const uint32_t *keys, const int64_t *weights, uint64_t n,
                          int64_t *sketch)
{
    for (int32_t t = 0; t < d; ++t) {
        for (uint64_t j = 0; j < m; ++j) {
            const uint64_t *a_tj = ams_coef + ((size_t)t * m + j) * n_edges * 4;
            int64_t sum = 0;
            for (uint64_t i = 0; i < n; ++i) {
                int64_t x = 1;
                for (int32_t col = 0; col < n_cols; ++col) {
                    uint32_t key = keys[i * (uint64_t)n_cols + col];
                    for (int32_t e = 0; e < col_nedges[col]; ++e)
                        x = or_sign(a_tj + 4 * col_edges[col * max_edges + e], key) * x;
                }
                int64_t delta = weights ? weights[i] : 1;
                sum = (int64_t)((uint64_t)sum + (uint64_t)x * (uint64_t)delta);
            }
            uint64_t *c = (uint64_t *)(sketch + (size_t)t * m + j);
            *c += (uint64_t)sum;
        }
    }
}
