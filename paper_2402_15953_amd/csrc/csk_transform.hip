// Power-of-two transforms over the sketches: the fp64 complex FFT used by the estimate
// (Alg. 3 evaluates cross-correlations through FFT / IFFT) and the number-theoretic
// transform (same structure, Montgomery arithmetic modulo a 31-bit prime) used for the
// exact modular evaluation.
//
// Lengths up to 4096 are done in one pass inside LDS.  Longer lengths m = N1 * N2 (N2 =
// 2^S, from 1024 to 4096, default_split_bits() or the tuned split) use the four-step decomposition
// (Bailey): element n = N2 n1 + n2.
//   forward: pass 1 transforms each column n2 over n1 (stride N2) and multiplies output
//            f1 by w_m^(f1 n2); pass 2 transforms each row over n2.  Position N2 f1 + f2
//            then holds frequency f = f1 + N1 f2 (no final transpose).
//   inverse: takes that permuted order back to natural order: row pass over f2 with
//            w_m^(-n2 f1) applied to output n2, then the column pass over f1.
// Inside LDS each tile is loaded in bit-reversed order and finished by radix-2
// decimation-in-time stages; twiddles come from host-computed tables.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "csk_internal.h"
#include "csk_rings.h"
#include "csk_transform.h"

namespace csk {

namespace {

// A block transforms one tile of TILE elements: the fp64 FFT with TILE / 4 threads (two
// butterflies per thread per stage; the pass is bound by memory and wants the loads of
// many wavefronts), the NTT with TILE / 8 (four per thread: its passes wait on their
// barriers, and two independent butterfly groups per thread between two barriers
// measured 13-20% faster than one; four per thread were slower again).  Two-pass lengths use the smallest tile that keeps the column
// pass's reads in runs of at least 8 elements: a 2^16-point transform is 64 blocks of
// 1024 elements per vector (24 KB of LDS each, several blocks per CU) rather than 16
// blocks of 4096 (96 KB, one per CU), so its passes fill the chip.
constexpr int kSingleTile = 4096;

// LDS position of tile element i: one padding word after every 32, so that the
// bit-reversed loads (whose first 64 positions are multiples of the tile length / 64)
// and the butterflies at small strides spread over the banks instead of meeting on a
// few of them.
__device__ __forceinline__ int lp(int i) { return i + (i >> 5); }
template <int TILE>
constexpr int lds_len() { return TILE + TILE / 32; }

__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits)
{
    return bits ? (__brev(x) >> (32 - bits)) : 0u;
}

// Copies w_L^j (j < L / 2, L = 2^log2L) from the table tw[k] = w_T^k, T = 2^log2T, into
// LDS; every stage of a length-L transform takes its twiddles from there.
template <int NT, class T>
__device__ __forceinline__ void load_stage_twiddles(T *stw, int log2L, const T *__restrict__ tw, int log2T)
{
    for (int j = threadIdx.x; j < (1 << (log2L - 1)); j += NT) stw[j] = tw[(size_t)j << (log2T - log2L)];
}

// Radix-2 DIT stages on C interleaved transforms of length 2^log2L held in LDS as
// s[lp(n * C + c)] (bit-reversed input, natural output); stw from load_stage_twiddles.
// Stages go in pairs: a thread takes the four elements two consecutive stages combine,
// applies both stages' radix-2 butterflies in registers (the same operations as two
// separate stages, so the same rounding), and writes them back once.
//
// Addressing: with D = half * C the tile distance between a group's elements, group b
// starts at idx0 = ((b >> log2 D) << (log2 D + 2)) + (b & (D - 1)), and its block of 4D
// tile positions starts at a multiple of 4D.  A power-of-two block of at most 32
// positions then lies inside one 32-position stretch, and larger ones start on one, so
// element j sits jD + (jD >> 5) padded positions after element 0 for every group: one
// padded address per group, the other three at offsets uniform over the stage.
template <int NT, class Ring>
__device__ __forceinline__ void lds_stages(typename Ring::T *s, int log2L, int log2C, const Ring &R,
                                           const typename Ring::T *stw)
{
    using T = typename Ring::T;
    int lh = 0;
    for (; lh + 1 < log2L; lh += 2) {
        const int sD = lh + log2C;
        const int D = 1 << sD;
        const int o1 = D + (D >> 5), o2 = 2 * D + ((2 * D) >> 5), o3 = 3 * D + ((3 * D) >> 5);
        const int sh2 = log2L - lh - 2;           // twiddle index shift of the second stage
        const int quarter = 1 << (log2L - 2);     // (k + half) << sh2 = (k << sh2) + quarter
        const int kmask = (1 << lh) - 1;
        const int ngr = (1 << (log2L - 2)) << log2C;
        for (int b = threadIdx.x; b < ngr; b += NT) {
            T *e = s + lp(((b >> sD) << (sD + 2)) + (b & (D - 1)));
            const int w2i = ((b >> log2C) & kmask) << sh2;
            const T x0 = e[0], x1 = e[o1], x2 = e[o2], x3 = e[o3];
            // stage lh: pairs (0, 1) and (2, 3), twiddle w_{2 half}^k
            const T w1 = stw[w2i << 1];
            T v = R.mul(x1, w1);
            const T y0 = R.add(x0, v), y1 = R.sub(x0, v);
            v = R.mul(x3, w1);
            const T y2 = R.add(x2, v), y3 = R.sub(x2, v);
            // stage lh + 1: pairs (0, 2) with w_{4 half}^k and (1, 3) with w_{4 half}^(k + half)
            const T w2 = stw[w2i];
            const T w3 = stw[w2i + quarter];
            v = R.mul(y2, w2);
            e[0] = R.add(y0, v);
            e[o2] = R.sub(y0, v);
            v = R.mul(y3, w3);
            e[o1] = R.add(y1, v);
            e[o3] = R.sub(y1, v);
        }
        __syncthreads();
    }
    for (; lh < log2L; ++lh) {  // the last stage when their number is odd
        const int sD = lh + log2C;
        const int D = 1 << sD;
        const int o1 = D + (D >> 5);
        const int sh = log2L - lh - 1;
        const int kmask = (1 << lh) - 1;
        const int nbf = (1 << (log2L - 1)) << log2C;
        for (int b = threadIdx.x; b < nbf; b += NT) {
            T *e = s + lp(((b >> sD) << (sD + 1)) + (b & (D - 1)));
            const T u = e[0];
            const T v = R.mul(e[o1], stw[((b >> log2C) & kmask) << sh]);
            e[0] = R.add(u, v);
            e[o1] = R.sub(u, v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- fp64 complex FFT pass

// Source of a pass: either the complex work buffer, or (first pass) the int64 sketches
// of the (relation, repetition) pair packed into one complex vector: re + i * im.
struct F64Src {
    const int64_t *const *re;  // [n_vec] sketch loaded as the real part (null: in place)
    const int64_t *const *im;  // [n_vec] sketch loaded as the imaginary part (entry null: 0)
};

template <int TILE>
__global__ __launch_bounds__(TILE / 4) void k_fft_f64(F64Src src, double2 *buf, PassGeom g,
                                                     const double2 *__restrict__ tw, int log2T)
{
    constexpr int NT = TILE / 4;
    __shared__ double2 s[lds_len<TILE>()];
    __shared__ double2 stw[TILE / 2];
    const int v = blockIdx.x;
    const int blk = blockIdx.y;
    const int C = 1 << g.log2C;
    const int L = 1 << g.log2L;
    const int64_t m = (int64_t)1 << g.log2m;
    const int64_t base = (int64_t)blk * g.block_stride;
    double2 *vec = buf + (size_t)v * m;
    const int total = L << g.log2C;
    if (src.re) {
        const int64_t *re = src.re[v];
        const int64_t *im = src.im[v];
        for (int idx = threadIdx.x; idx < total; idx += NT) {
            const int n = idx >> g.log2C, c = idx & (C - 1);
            const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
            s[lp((bitrev(n, g.log2L) << g.log2C) + c)] =
                make_double2((double)re[pos], im ? (double)im[pos] : 0.0);
        }
    } else {
        for (int idx = threadIdx.x; idx < total; idx += NT) {
            const int n = idx >> g.log2C, c = idx & (C - 1);
            const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
            s[lp((bitrev(n, g.log2L) << g.log2C) + c)] = vec[pos];
        }
    }
    load_stage_twiddles<NT>(stw, g.log2L, tw, log2T);
    __syncthreads();
    RingC R;
    lds_stages<NT, RingC>(s, g.log2L, g.log2C, R, stw);
    for (int idx = threadIdx.x; idx < total; idx += NT) {
        const int n = idx >> g.log2C, c = idx & (C - 1);
        const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
        double2 val = s[lp((n << g.log2C) + c)];
        if (g.twiddle) {
            const int64_t colid = (int64_t)blk * C + c;
            const int64_t e = ((int64_t)n * colid) & (m - 1);
            val = R.mul(val, tw[(size_t)e << (log2T - g.log2m)]);
        }
        vec[pos] = val;
    }
}

// ---------------------------------------------------------------- NTT pass

struct ModSrc {
    const int64_t *const *ptr;  // [vec_per_prime] sketch of vector v % vec_per_prime (null: in place)
};

template <int TILE, int NT>
__global__ __launch_bounds__(NT) void k_ntt(ModSrc src, uint32_t *buf, PassGeom g, int vec_per_prime,
                                           const PrimeDev *__restrict__ primes,
                                           const uint32_t *__restrict__ roots, int log2T, int inverse,
                                           const int32_t *__restrict__ rep_of, const int32_t *__restrict__ kp)
{
    __shared__ uint32_t s[lds_len<TILE>()];
    __shared__ uint32_t stw[TILE / 2];
    __shared__ uint32_t s_row[64];  // row passes with twiddles: w^(j blk), j < 64
    const int v = blockIdx.x;
    const int pi = v / vec_per_prime;
    if (kp && pi >= kp[rep_of[v % vec_per_prime]]) return;  // prime not needed
    const PrimeDev &P = primes[pi];  // by reference: a copy with minv[] indexed would live in scratch
    const RingM R{P.p, P.pinv_neg};
    const uint32_t *tw = roots + ((size_t)(2 * pi + inverse) << log2T);
    const int blk = blockIdx.y;
    const int C = 1 << g.log2C;
    const int L = 1 << g.log2L;
    const int64_t m = (int64_t)1 << g.log2m;
    const int64_t base = (int64_t)blk * g.block_stride;
    uint32_t *vec = buf + (size_t)v * m;
    const int total = L << g.log2C;
    if (src.ptr) {
        const int64_t *in = src.ptr[v % vec_per_prime];
        for (int idx = threadIdx.x; idx < total; idx += NT) {
            const int n = idx >> g.log2C, c = idx & (C - 1);
            const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
            s[lp((bitrev(n, g.log2L) << g.log2C) + c)] = mont_from_i64(R, in[pos], P.r2, P.r3, P.neg2_64);
        }
    } else {
        for (int idx = threadIdx.x; idx < total; idx += NT) {
            const int n = idx >> g.log2C, c = idx & (C - 1);
            const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
            s[lp((bitrev(n, g.log2L) << g.log2C) + c)] = vec[pos];
        }
    }
    load_stage_twiddles<NT>(stw, g.log2L, tw, log2T);
    if (g.twiddle && g.log2C == 0 && threadIdx.x < 64)
        s_row[threadIdx.x] = tw[(size_t)(((int64_t)threadIdx.x * blk) & (m - 1)) << (log2T - g.log2m)];
    __syncthreads();
    lds_stages<NT, RingM>(s, g.log2L, g.log2C, R, stw);
    for (int idx = threadIdx.x; idx < total; idx += NT) {
        const int n = idx >> g.log2C, c = idx & (C - 1);
        const int64_t pos = base + (int64_t)c * g.col_stride + (int64_t)n * g.elem_stride;
        uint32_t val = s[lp((n << g.log2C) + c)];
        if (g.twiddle) {
            const int sh = log2T - g.log2m;
            if (g.log2C > 0) {
                // w^(n (blk C + c)) = w^(n blk C) w^(n c): the first factor is one entry
                // for the C lanes of one n, the second lies in the table's first L C
                // entries (n c < L C), so neither is a scattered read of a table of m
                // entries (exact arithmetic: the same residue as one lookup)
                const uint32_t a = tw[(size_t)(((int64_t)n * blk * C) & (m - 1)) << sh];
                const uint32_t b = tw[(size_t)((int64_t)n * c) << sh];
                val = R.mul(R.mul(val, a), b);
            } else {
                // a row (C = 1): w^(n blk) = w^(64 (n >> 6) blk) w^((n & 63) blk), the
                // first factor one entry for a wavefront's 64 lanes, the second from LDS
                const uint32_t a = tw[(size_t)(((int64_t)(n >> 6) * 64 * blk) & (m - 1)) << sh];
                val = R.mul(R.mul(val, a), s_row[n & 63]);
            }
        }
        if (g.scale) val = R.mul(val, P.minv[g.log2m]);
        vec[pos] = val;
    }
}

// Two-pass lengths: tiles of N2 = 2^S elements, columns of N1 = 2^(log2m - S) <= N2.
PassGeom column_pass(int log2m, int S, bool twiddle)
{
    PassGeom g{};
    g.log2m = log2m;
    g.log2L = log2m - S;
    g.log2C = S - g.log2L;
    g.elem_stride = (int64_t)1 << S;
    g.col_stride = 1;
    g.block_stride = (int64_t)1 << g.log2C;
    g.blocks = (1 << S) >> g.log2C;
    g.twiddle = twiddle;
    return g;
}

PassGeom row_pass(int log2m, int S, bool twiddle)
{
    PassGeom g{};
    g.log2m = log2m;
    g.log2L = S;
    g.log2C = 0;
    g.elem_stride = 1;
    g.col_stride = 0;
    g.block_stride = (int64_t)1 << S;
    g.blocks = 1 << (log2m - S);
    g.twiddle = twiddle;
    return g;
}

// Launch of one pass with the tile its geometry needs (single pass: the whole vector in
// one 4096-element tile; two-pass lengths: 2^S elements).
template <class F>
void with_tile(const PassGeom &g, bool single, F &&f)
{
    const int tile_bits = g.log2L + g.log2C;  // = S for both passes
    if (single || tile_bits == 12) f(std::integral_constant<int, kSingleTile>{});
    else if (tile_bits == 10) f(std::integral_constant<int, 1024>{});
    else f(std::integral_constant<int, 2048>{});
}

PassGeom single_pass(int log2m)
{
    PassGeom g{};
    g.log2m = log2m;
    g.log2L = log2m;
    g.log2C = 0;
    g.elem_stride = 1;
    g.block_stride = 0;
    g.blocks = 1;
    return g;
}

}  // namespace

int split_for(int device, int log2m)
{
    const int t = tune_split(device, log2m);
    return t && split_ok(log2m, t) ? t : default_split_bits(log2m);
}

cs_status fft_f64_forward(const int64_t *const *re, const int64_t *const *im, int n_vec, double2 *buf, int log2m,
                          int S, const double2 *tw, int log2T, hipStream_t s)
{
    if (n_vec == 0) return CS_OK;
    F64Src first{re, im};
    F64Src self{nullptr, nullptr};
    auto pass = [&](const PassGeom &g, bool single, const F64Src &src) {
        with_tile(g, single, [&](auto tile) {
            constexpr int T = decltype(tile)::value;
            hipLaunchKernelGGL(k_fft_f64<T>, dim3(n_vec, g.blocks), dim3(T / 4), 0, s, src, buf, g, tw, log2T);
        });
        return hipGetLastError();
    };
    if (log2m <= 12) {
        CSK_HIP(pass(single_pass(log2m), true, first));
        return CS_OK;
    }
    CSK_HIP(pass(column_pass(log2m, S, true), false, first));
    CSK_HIP(pass(row_pass(log2m, S, false), false, self));
    return CS_OK;
}

namespace {
// The column pass of the NTT reads its columns in runs of C 4-byte residues; with the
// split shared with the fp64 FFT (runs of >= 8 complex doubles = 128 bytes) C can be as
// low as 8 (32 bytes), so NTT column passes take up to 32 columns per block (tiles up
// to 16384 residues, 64 KB of LDS, 1024 threads).  The decomposition, and with it the
// output order, is unchanged.
PassGeom widen_columns(PassGeom g)
{
    while (g.log2C < 5 && g.blocks > 1 && g.log2L + g.log2C < 14) {
        ++g.log2C;
        g.block_stride <<= 1;
        g.blocks >>= 1;
    }
    return g;
}

hipError_t ntt_pass(const PassGeom &g, bool single, const ModSrc &src, int n_vec, uint32_t *buf, int vec_per_prime,
                    const PrimeDev *primes, const uint32_t *roots, int log2T, int inverse, const int32_t *rep_of,
                    const int32_t *kp, hipStream_t s)
{
    auto go = [&](auto tile) {
        constexpr int T = decltype(tile)::value;
        constexpr int NT = T / 8 < 1024 ? T / 8 : 1024;
        hipLaunchKernelGGL((k_ntt<T, NT>), dim3(n_vec, g.blocks), dim3(NT), 0, s, src, buf, g, vec_per_prime,
                           primes, roots, log2T, inverse, rep_of, kp);
    };
    const int tile_bits = g.log2L + g.log2C;
    if (single) go(std::integral_constant<int, kSingleTile>{});
    else if (tile_bits <= 10) go(std::integral_constant<int, 1024>{});
    else if (tile_bits == 11) go(std::integral_constant<int, 2048>{});
    else if (tile_bits == 12) go(std::integral_constant<int, 4096>{});
    else if (tile_bits == 13) go(std::integral_constant<int, 8192>{});
    else go(std::integral_constant<int, 16384>{});
    return hipGetLastError();
}
}  // namespace

cs_status ntt_forward(const int64_t *const *ptrs, int vec_per_prime, int n_primes, uint32_t *buf, int log2m, int S,
                      const PrimeDev *primes, const uint32_t *roots, int log2T, hipStream_t s,
                      const int32_t *rep_of, const int32_t *kp)
{
    const int n_vec = vec_per_prime * n_primes;
    if (n_vec == 0) return CS_OK;
    ModSrc first{ptrs};
    ModSrc self{nullptr};
    const ModSrc &in = ptrs ? first : self;
    if (log2m <= 12) {
        CSK_HIP(ntt_pass(single_pass(log2m), true, in, n_vec, buf, vec_per_prime, primes, roots, log2T, 0, rep_of,
                         kp, s));
        return CS_OK;
    }
    CSK_HIP(ntt_pass(widen_columns(column_pass(log2m, S, true)), false, in, n_vec, buf, vec_per_prime, primes,
                     roots, log2T, 0, rep_of, kp, s));
    CSK_HIP(ntt_pass(row_pass(log2m, S, false), false, self, n_vec, buf, vec_per_prime, primes, roots, log2T, 0,
                     rep_of, kp, s));
    return CS_OK;
}

cs_status ntt_inverse(int vec_per_prime, int n_primes, uint32_t *buf, int log2m, int S, const PrimeDev *primes,
                      const uint32_t *roots, int log2T, hipStream_t s)
{
    const int n_vec = vec_per_prime * n_primes;
    if (n_vec == 0) return CS_OK;
    ModSrc self{nullptr};
    if (log2m <= 12) {
        PassGeom g = single_pass(log2m);
        g.scale = 1;
        CSK_HIP(ntt_pass(g, true, self, n_vec, buf, vec_per_prime, primes, roots, log2T, 1, nullptr, nullptr, s));
        return CS_OK;
    }
    CSK_HIP(ntt_pass(row_pass(log2m, S, true), false, self, n_vec, buf, vec_per_prime, primes, roots, log2T, 1,
                     nullptr, nullptr, s));
    PassGeom g2 = widen_columns(column_pass(log2m, S, false));
    g2.scale = 1;
    CSK_HIP(ntt_pass(g2, false, self, n_vec, buf, vec_per_prime, primes, roots, log2T, 1, nullptr, nullptr, s));
    return CS_OK;
}

}  // namespace csk
