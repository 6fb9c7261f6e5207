// Join-size estimate (Eq. 5 evaluated as in Alg. 3) and the median over repetitions.
//
// Plans (chosen from the join graph at create time):
//   DOT       two relations, one join: X_t = sum_j c_0[t][j] c_1[t][j] (the Count-sketch
//             inner product), exact in 128-bit integers.
//   SPECTRAL  every graph component joins exactly two attributes.  Substituting the
//             inverse DFT of every sketch into Eq. 5 and summing over the component
//             indices leaves one frequency per relation tied to its neighbours' with
//             opposite sign, so X_t = (1/m) sum_f prod_k C_k[f], with C_k the DFT of
//             c_k[t] conjugated on alternate levels of the relation tree (for a chain:
//             conj(C_0) C_1 conj(C_2) ...).  This is Alg. 3's sequence of
//             cross-correlations and Hadamard products followed by SumElements, taken
//             entirely in the frequency domain.  Computed with the fp64 FFT; a certified
//             a-priori bound B_t on |fp64 result - X_t| decides whether rounding gives
//             the exact integer; otherwise the residues of X_t modulo enough NTT primes
//             (the same product-reduce in modular arithmetic) select the unique integer
//             within B_t of the fp64 value.
//   GENERAL   some component joins three or more attributes: Alg. 3's register program
//             (Hadamard products, cross-correlations through NTT / inverse NTT) in
//             modular arithmetic for enough primes to cover |X_t| <= prod_k ||c_k||_1,
//             then the Chinese remainder theorem.
// The median (lower middle element for even d) is taken on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "csk_handle.h"
#include "csk_rings.h"
#include "csk_transform.h"

namespace csk {

namespace {

constexpr int kThreads = 256;

struct RepDev {
    double xf;       // fp64 estimate from the FFT (spectral plan)
    double bound;    // certified bound on |xf - X_t|
    double value;    // final fp64 value
    int64_t lo, hi;  // exact X_t as int128 when exact
    int32_t exact;
    int32_t kprimes; // primes the modular step must use for this repetition
    int32_t status;  // 1: value beyond the exact range
    int32_t window;  // spectral plan: residues select X within bound of rint(xf)
};

struct OutDev {
    double value;
    int64_t lo, hi;
    int32_t exact, fits, n_modular, median_rep;
};

struct CrtTables {
    uint32_t p[kMaxPrimes];
    uint32_t inv[kMaxPrimes][kMaxPrimes];     // inv[j][i] = p_j^-1 mod p_i
    uint32_t half[kMaxPrimes][kMaxPrimes];    // half[K-1]: digits of (P_K - 1) / 2
    double log2p[kMaxPrimes];
};

// ---------------------------------------------------------------- small helpers

__device__ __forceinline__ double warp_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Butterfly reductions: every lane ends with the same value (fixed order).
__device__ __forceinline__ double wave_allsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_allmax(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide sum with a fixed reduction order.
__device__ double block_sum(double v, double *sh)
{
    v = warp_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;  // valid in thread 0
}

__device__ double block_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
    return r;
}

// Correctly rounded conversion of a signed 128-bit integer to double.
__device__ double i128_to_double(__int128 x)
{
    const bool neg = x < 0;
    unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)x : (unsigned __int128)x;
    const uint64_t hi = (uint64_t)(u >> 64);
    double r;
    if (hi == 0) {
        r = (double)(uint64_t)u;
    } else {
        const int b = 127 - __clzll(hi);  // top bit position, >= 64
        const int sh = b - 63;
        const unsigned __int128 mask = (((unsigned __int128)1) << sh) - 1;
        uint64_t t = (uint64_t)(u >> sh);
        if (u & mask) t |= 1;  // sticky bit keeps round-to-nearest-even exact
        r = ldexp((double)t, sh);
    }
    return neg ? -r : r;
}

// Integer-valued double (|x| < 2^126) to int128.
__device__ __int128 double_to_i128(double x)
{
    if (fabs(x) < 0x1p62) return (__int128)(int64_t)x;
    int e;
    const double f = frexp(x, &e);            // x = f * 2^e, 0.5 <= |f| < 1, e >= 63
    const int64_t mant = (int64_t)ldexp(f, 53);
    const bool neg = mant < 0;
    unsigned __int128 u = (unsigned __int128)(uint64_t)(neg ? -mant : mant) << (e - 53);
    return neg ? -(__int128)u : (__int128)u;
}

__device__ uint32_t mod_u128(unsigned __int128 u, uint32_t p)
{
    uint64_t r = 0;
    for (int i = 3; i >= 0; --i) {
        const uint32_t limb = (uint32_t)(u >> (32 * i));
        r = ((r << 32) | limb) % p;
    }
    return (uint32_t)r;
}

__device__ uint32_t mod_i128(__int128 x, uint32_t p)
{
    if (x >= 0) return mod_u128((unsigned __int128)x, p);
    const uint32_t r = mod_u128((unsigned __int128)0 - (unsigned __int128)x, p);
    return r ? p - r : 0;
}

__device__ void garner(const uint32_t *res, int K, const CrtTables &T, uint32_t *dig)
{
    for (int i = 0; i < K; ++i) {
        const uint64_t pi = T.p[i];
        uint64_t x = res[i] % pi;
        for (int j = 0; j < i; ++j) {
            const uint64_t dj = dig[j] % pi;
            x = (x + pi - dj) % pi;
            x = (x * T.inv[j][i]) % pi;
        }
        dig[i] = (uint32_t)x;
    }
}

// Mixed-radix digits -> centered integer.  Returns false unless |X| < ~2^126.
__device__ bool digits_to_i128(const uint32_t *dig, int K, const CrtTables &T, __int128 *out, double *dval)
{
    bool upper = false;
    for (int i = K - 1; i >= 0; --i) {
        if (dig[i] != T.half[K - 1][i]) {
            upper = dig[i] > T.half[K - 1][i];
            break;
        }
    }
    uint32_t w[kMaxPrimes];
    for (int i = 0; i < K; ++i) w[i] = upper ? T.p[i] - 1 - dig[i] : dig[i];
    if (upper) {  // P - X' = (P - 1 - X') + 1
        for (int i = 0; i < K; ++i) {
            if (w[i] + 1 < T.p[i]) {
                w[i] += 1;
                break;
            }
            w[i] = 0;
        }
    }
    double dv = 0.0;
    for (int i = K - 1; i >= 0; --i) dv = dv * (double)T.p[i] + (double)w[i];
    *dval = upper ? -dv : dv;
    // |X| < 2^126 is guaranteed representable: refuse a multiply once acc >= 2^95
    // (acc * p + w < 2^95 * 2^31 + 2^31 <= 2^126 + 2^31).
    unsigned __int128 acc = 0;
    for (int i = K - 1; i >= 0; --i) {
        if ((acc >> 95) != 0) return false;
        acc = acc * T.p[i] + w[i];
    }
    *out = upper ? -(__int128)acc : (__int128)acc;
    return true;
}

// ---------------------------------------------------------------- descriptors

// One sketch vector c_k[t] (norm partials at off * 2 doubles).
struct SkDesc {
    const int64_t *p;
    int32_t log2m;
    int32_t nb;
    int64_t off;
    uint32_t m;
    uint32_t pad;
};

// One repetition t of query q.
struct RepDesc {
    const int64_t *c0;     // DOT plan: relation 0 and 1 at repetition t
    const int64_t *c1;
    int32_t q, t, log2m, r, d;
    int32_t S;             // row length 2^S of the two-pass transforms of this length
    uint32_t m;            // buckets (log2m is exact only for powers of two)
    uint32_t conj;         // SPECTRAL: relations taken conjugated
    int32_t vec_base;      // SPECTRAL: first packed vector of query q in its group's buffer
    int32_t nb;            // blocks of this repetition's reductions
    int32_t sk_base;       // first sketch (k * d + t order) of query q in the SkDesc table
    int32_t mod_vec_base;  // modular pass: first vector of query q in its group's buffer
    int64_t spec_off;      // fp64 spectral partials, (2 + r) doubles per block
    int64_t dot_off;       // DOT partials, 4 words per block (int128 sum, fp64 sum, fp64 sum of |terms|)
    int64_t mod_off;       // modular partials (per prime plane)
};

struct QDesc {
    int32_t plan, r, d, log2m, rep_base, nb;
    uint32_t m;
    // where this query's partials start (its first sketch's norm pair, its first
    // repetition's spectral sums and residues): the finalize reads them without going
    // through the repetition and sketch descriptors first
    int64_t norm_off0, spec_off0, mod_off0;
};

// ---------------------------------------------------------------- kernels

// Flattened launches: block b belongs to item i with prefix[i] <= b < prefix[i + 1].
__device__ __forceinline__ int find_item(const int64_t *__restrict__ prefix, int n, int64_t b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Sum of squares and of absolute values of each sketch vector (fp64), per block.
__global__ __launch_bounds__(kThreads) void k_norms(const SkDesc *__restrict__ sks, const int64_t *__restrict__ prefix,
                                                    int n_items, double *partials)
{
    __shared__ double sh[kThreads / 64];
    const int item = find_item(prefix, n_items, blockIdx.x);
    const SkDesc S = sks[item];
    const int blk = (int)(blockIdx.x - prefix[item]);
    const int64_t m = S.m;
    double s2 = 0.0, s1 = 0.0;
    for (int64_t j = (int64_t)blk * kThreads + threadIdx.x; j < m; j += (int64_t)S.nb * kThreads) {
        const double v = (double)S.p[j];
        s2 += v * v;
        s1 += fabs(v);
    }
    const double a = block_sum(s2, sh);
    const double b = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        double *o = partials + (S.off + blk) * 2;
        o[0] = a;
        o[1] = b;
    }
}

// 128-bit inner product of c_0[t] and c_1[t], per block, wrapping modulo 2^128, with
// an fp64 sum of the products and an fp64 sum of their absolute values beside it: the
// latter bounds every partial sum, so the finalize knows whether the wrapped integer is
// the true one (the sum of |terms| stays below 2^126).
__global__ __launch_bounds__(kThreads) void k_dot(const RepDesc *__restrict__ reps, const int32_t *__restrict__ idx,
                                                  const int64_t *__restrict__ prefix, int n_items,
                                                  unsigned long long *partials)
{
    __shared__ unsigned __int128 sh[kThreads];
    __shared__ double shf[kThreads / 64];
    const int item = find_item(prefix, n_items, blockIdx.x);
    const RepDesc D = reps[idx[item]];
    const int blk = (int)(blockIdx.x - prefix[item]);
    const int64_t m = D.m;
    __int128 acc = 0;
    double fs = 0.0, fa = 0.0;
    for (int64_t j = (int64_t)blk * kThreads + threadIdx.x; j < m; j += (int64_t)D.nb * kThreads) {
        const int64_t x = D.c0[j], y = D.c1[j];
        acc += (__int128)x * (__int128)y;
        const double p = (double)x * (double)y;
        fs += p;
        fa += fabs(p);
    }
    sh[threadIdx.x] = (unsigned __int128)acc;
    const double bs = block_sum(fs, shf);
    const double ba = block_sum(fa, shf);
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long *o = partials + (D.dot_off + blk) * 4;
        o[0] = (unsigned long long)(uint64_t)sh[0];
        o[1] = (unsigned long long)(uint64_t)(sh[0] >> 64);
        o[2] = (unsigned long long)__double_as_longlong(bs);
        o[3] = (unsigned long long)__double_as_longlong(ba);
    }
}

// fp64 spectral product-reduce for repetitions idx[blockIdx.y] of one m-group.
// Sketch s = k * d + t of a query is half (s & 1) of packed vector vec_base + s / 2.
// partials: sum Re(term), sum |Re|+|Im| of terms, max |C_k| per relation.
__global__ __launch_bounds__(kThreads) void k_spec_f64(const double2 *__restrict__ Z,
                                                       const RepDesc *__restrict__ reps,
                                                       const int32_t *__restrict__ idx,
                                                       const int64_t *__restrict__ prefix, int n_items,
                                                       double *partials)
{
    __shared__ double sh[kThreads / 64];
    const int item = find_item(prefix, n_items, blockIdx.x);
    const RepDesc D = reps[idx[item]];
    const int blk = (int)(blockIdx.x - prefix[item]);
    const int log2m = D.log2m, S = D.S;
    const uint32_t m = 1u << log2m;
    const int r = D.r;
    double acc = 0.0, acc_abs = 0.0;
    double mx[kMaxRel];
#pragma unroll
    for (int k = 0; k < kMaxRel; ++k) mx[k] = 0.0;
    for (uint32_t pos = blk * kThreads + threadIdx.x; pos < m; pos += (uint32_t)D.nb * kThreads) {
        const uint32_t f = pos_freq(pos, log2m, S);
        const uint32_t npos = freq_pos((m - f) & (m - 1), log2m, S);
        double pr = 1.0, pi = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxRel; ++k) {
            if (k < r) {
                const int sidx = k * D.d + D.t;
                const double2 *zv = Z + (size_t)(D.vec_base + (sidx >> 1)) * m;
                const double2 a = zv[pos], b = zv[npos];
                double cr, ci;
                if ((sidx & 1) == 0) {
                    cr = 0.5 * (a.x + b.x);
                    ci = 0.5 * (a.y - b.y);
                } else {
                    cr = 0.5 * (a.y + b.y);
                    ci = 0.5 * (b.x - a.x);
                }
                if ((D.conj >> k) & 1u) ci = -ci;
                mx[k] = fmax(mx[k], fabs(cr) + fabs(ci));
                const double nr = pr * cr - pi * ci;
                const double ni = pr * ci + pi * cr;
                pr = nr;
                pi = ni;
            }
        }
        acc += pr;
        acc_abs += fabs(pr) + fabs(pi);
    }
    double *o = partials + (D.spec_off + (int64_t)blk * (2 + r));
    const double s0 = block_sum(acc, sh);
    if (threadIdx.x == 0) o[0] = s0;
    const double s1 = block_sum(acc_abs, sh);
    if (threadIdx.x == 0) o[1] = s1;
    for (int k = 0; k < r; ++k) {
        const double mk = block_max(mx[k], sh);
        if (threadIdx.x == 0) o[2 + k] = mk;
    }
}

// Modular spectral product-reduce.  Buffer [K][vpp][m]; query q's sketch k * d + t is
// vector mod_vec_base + k * d + t.  partials [K][plane] at mod_off.
__global__ __launch_bounds__(kThreads) void k_spec_mod(const uint32_t *__restrict__ N, int vpp,
                                                       const RepDesc *__restrict__ reps,
                                                       const int32_t *__restrict__ idx,
                                                       const int64_t *__restrict__ prefix, int n_items,
                                                       const PrimeDev *__restrict__ primes, int64_t plane,
                                                       uint32_t *partials, const int32_t *__restrict__ kp)
{
    __shared__ uint32_t sh[kThreads];
    const int item = find_item(prefix, n_items, blockIdx.x);
    if (kp && (int)blockIdx.y >= kp[idx[item]]) return;  // prime not needed by this repetition
    const RepDesc D = reps[idx[item]];
    const int blk = (int)(blockIdx.x - prefix[item]);
    const int pi = blockIdx.y;
    const PrimeDev P = primes[pi];
    const RingM R{P.p, P.pinv_neg};
    const int log2m = D.log2m, S = D.S;
    const uint32_t m = 1u << log2m;
    const uint32_t *base = N + (size_t)pi * vpp * m;
    uint32_t acc = 0;
    // four positions per pass, their loads of one relation's factors issued together
    // (the sum is exact in Z_p, so its order does not matter)
    constexpr int U = 8;
    const uint32_t stride = (uint32_t)D.nb * kThreads;
    for (uint32_t p0 = blk * kThreads + threadIdx.x; p0 < m; p0 += U * stride) {
        uint32_t ps[U], nps[U], prod[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t q = p0 + u * stride;
            ps[u] = q < m ? q : 0u;  // a position past the end reads position 0 and is not added
            const uint32_t f = pos_freq(ps[u], log2m, S);
            nps[u] = freq_pos((m - f) & (m - 1), log2m, S);
            prod[u] = P.one;
        }
        for (int k = 0; k < D.r; ++k) {
            const uint32_t *v = base + (size_t)(D.mod_vec_base + k * D.d + D.t) * m;
            const bool cj = (D.conj >> k) & 1u;
            uint32_t val[U];
#pragma unroll
            for (int u = 0; u < U; ++u) val[u] = v[cj ? nps[u] : ps[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) prod[u] = R.mul(prod[u], val[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (p0 + u * stride < m) acc = R.add(acc, prod[u]);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = R.add(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(size_t)pi * plane + D.mod_off + blk] = sh[0];
}

// ---- general plan register operations, buffers [K][d][m] per register

__global__ void k_mod_load(uint32_t *reg, const int64_t *__restrict__ sk, uint32_t m, int d,
                           const PrimeDev *__restrict__ primes)
{
    const int v = blockIdx.y;  // i * d + t
    const PrimeDev P = primes[v / d];
    const RingM R{P.p, P.pinv_neg};
    const int64_t *c = sk + (size_t)(v % d) * m;
    uint32_t *o = reg + (size_t)v * m;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        o[j] = mont_from_i64(R, c[j], P.r2, P.r3, P.neg2_64);
}

__global__ void k_mod_ones(uint32_t *reg, uint32_t m, int d, const PrimeDev *__restrict__ primes)
{
    const int v = blockIdx.y;
    const uint32_t one = primes[v / d].one;
    uint32_t *o = reg + (size_t)v * m;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        o[j] = one;
}

// dst = dst o src (time domain) or dst[pos] = src[-f] * dst[f] (frequency domain, the
// pointwise step of the cross-correlation src star dst).
__global__ void k_mod_mul(uint32_t *dst, const uint32_t *__restrict__ src, uint32_t m, int log2m, int S, int d,
                          const PrimeDev *__restrict__ primes, int negate_src)
{
    const int v = blockIdx.y;
    const PrimeDev P = primes[v / d];
    const RingM R{P.p, P.pinv_neg};
    uint32_t *o = dst + (size_t)v * m;
    const uint32_t *a = src + (size_t)v * m;
    for (uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x; pos < m; pos += gridDim.x * blockDim.x) {
        uint32_t sp = pos;
        if (negate_src) sp = freq_pos((m - pos_freq(pos, log2m, S)) & (m - 1), log2m, S);
        o[pos] = R.mul(o[pos], a[sp]);
    }
}

// Sum of register vector (prime i, repetition t) -> partials[i * plane + mod_off(rep) + b].
__global__ __launch_bounds__(kThreads) void k_mod_sum(const uint32_t *__restrict__ reg, uint32_t m, int d,
                                                      const PrimeDev *__restrict__ primes, int nb,
                                                      const RepDesc *__restrict__ reps, int rep_base,
                                                      int64_t plane, uint32_t *partials)
{
    __shared__ uint32_t sh[kThreads];
    const int v = blockIdx.y;  // i * d + t
    const int pi = v / d, t = v % d;
    const PrimeDev P = primes[pi];
    const RingM R{P.p, P.pinv_neg};
    const uint32_t *a = reg + (size_t)v * m;
    uint32_t acc = 0;
    for (uint32_t j = blockIdx.x * kThreads + threadIdx.x; j < m; j += (uint32_t)nb * kThreads) acc = R.add(acc, a[j]);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = R.add(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[(size_t)pi * plane + reps[rep_base + t].mod_off + blockIdx.x] = sh[0];
}

// Zero-padded copy of length-m register vectors into length-M buffers (M >= 2m - 1, a
// power of two), reversed (i -> (m - i) mod m) when `reverse`: the operands of a linear
// convolution whose wrap-around sum is the cross-correlation of Def. 3.1 for any m.
__global__ void k_mod_pad(uint32_t *out, const uint32_t *__restrict__ in, uint32_t m, uint32_t M, int reverse)
{
    const int v = blockIdx.y;
    const uint32_t *a = in + (size_t)v * m;
    uint32_t *o = out + (size_t)v * M;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) {
        uint32_t val = 0;
        if (i < m) val = a[reverse ? (i == 0 ? 0 : m - i) : i];
        o[i] = val;
    }
}

// dst[j] = lin[j] + lin[j + m]: the circular (length m) result of a linear one.
__global__ void k_mod_fold(uint32_t *dst, const uint32_t *__restrict__ lin, uint32_t m, uint32_t M, int d,
                           const PrimeDev *__restrict__ primes)
{
    const int v = blockIdx.y;
    const PrimeDev &P = primes[v / d];
    const RingM R{P.p, P.pinv_neg};
    const uint32_t *l = lin + (size_t)v * M;
    uint32_t *o = dst + (size_t)v * m;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x)
        o[j] = j + m < M ? R.add(l[j], l[j + m]) : l[j];
}

// ---- finalize: one workgroup per query, one thread per repetition

struct FinalizeArgs {
    int32_t stage;        // 1: after the fp64 / dot / norms pass; 2: after the modular pass
    const QDesc *qs;
    const RepDesc *reps;
    const SkDesc *sks;
    const double *norms;
    const double *spec;
    const unsigned long long *dot;
    const uint32_t *modp;
    int64_t mod_plane;
    const PrimeDev *primes;
    CrtTables crt;
    RepDev *rs;
    OutDev *outs;
    int32_t *kp;    // stage 1 also stores each repetition's prime count here
    int32_t kcap;   // stage 2 finishes repetitions needing at most kcap primes
};

// A finalize block per query: 1024 threads (16 wavefronts, so each reduces one or two
// partial sets and the chains of dependent loads are short) when the queries fit one
// round of blocks, 256 for large batches.
constexpr int kFinThreadsFew = 1024, kFinThreadsMany = 256;
constexpr int kStage = kMaxD * 3 * kMaxRel;  // doubles of per-repetition bound terms
constexpr int kSpecPrimes = 5;                       // speculative modular step: primes (155 bits)
constexpr size_t kSpecBudget = (size_t)1 << 30;      // and its largest workspace
constexpr int kOverlapPrimes = 3;                    // at most this many: beside the fp64 chain
constexpr size_t kOverlapMinResidues = (size_t)1 << 24;  // and at least this many residues

// STAGE 1: fp64 / dot / norms pass; 2: residues of the modular pass; 3: both in one
// launch (the speculative residues were computed beside the fp64 pass).
template <int STAGE, int NT>
__global__ __launch_bounds__(NT) void k_finalize(FinalizeArgs a)
{
    __shared__ double s_val[kMaxD];
    __shared__ int64_t s_lo[kMaxD], s_hi[kMaxD];
    __shared__ int32_t s_ex[kMaxD], s_kp[kMaxD];
    // stage 1: per-block partials of this query reduced once, one wavefront per
    // sketch (norms) or repetition (spectral sums), in a fixed order
    __shared__ double s_q2[kMaxRel * kMaxD], s_l1[kMaxRel * kMaxD];
    __shared__ double s_sum[kMaxD], s_sabs[kMaxD], s_mx[kMaxD * kMaxRel];
    __shared__ double s_stage[kStage];  // scratch of the bound computation
    __shared__ uint32_t s_res[kMaxD * kMaxPrimes], s_dig[kMaxD * kMaxPrimes];
    const QDesc Q = a.qs[blockIdx.x];
    const int t = threadIdx.x;
    const double u = 0x1p-53;
    const double m = (double)Q.m;
    const int plan = Q.plan;
    const int wv = t >> 6, lane = t & 63;
    constexpr int kWaves = NT / 64;
    if (STAGE != 2 && plan != CS_PLAN_DOT) {
        // The nb <= 64 block partials of each owner (a sketch for the norms, a repetition
        // for the spectral sums) are reduced by one wavefront: lane b loads partial b and
        // a shuffle tree of depth 6 adds them, in a fixed order.
        const int nb = Q.nb;
        const int n_sk = Q.r * Q.d;
        const double *nrm = a.norms + Q.norm_off0 * 2;
        for (int o = wv; o < n_sk; o += kWaves) {
            double q2 = 0.0, l1 = 0.0;
            if (lane < nb) {
                const double *p = nrm + ((int64_t)o * nb + lane) * 2;
                q2 = p[0];
                l1 = p[1];
            }
            q2 = warp_sum(q2);
            l1 = warp_sum(l1);
            if (lane == 0) {
                s_q2[o] = q2;
                s_l1[o] = l1;
            }
        }
        if (plan == CS_PLAN_SPECTRAL) {
            const int w = 2 + Q.r;
            const double *spc = a.spec + Q.spec_off0;
            for (int o = wv; o < Q.d; o += kWaves) {
                const double *p = spc + ((int64_t)o * nb + lane) * w;
                double sm = lane < nb ? p[0] : 0.0, sa = lane < nb ? p[1] : 0.0;
                sm = warp_sum(sm);
                sa = warp_sum(sa);
                if (lane == 0) {
                    s_sum[o] = sm;
                    s_sabs[o] = sa;
                }
                for (int k = 0; k < Q.r; ++k) {
                    const double mk = wave_allmax(lane < nb ? p[2 + k] : 0.0);
                    if (lane == 0) s_mx[o * kMaxRel + k] = mk;
                }
            }
        }
    }
    if constexpr (STAGE != 1) {
        // residues: the nb partials of each (repetition, prime) summed by one wavefront
        // (stage 3: every prime of the speculative pass, the repetition's count not
        // being known yet)
        for (int o = wv; o < Q.d && (STAGE == 2 || plan == CS_PLAN_SPECTRAL); o += kWaves) {
            const int K = STAGE == 3 ? a.kcap : a.rs[Q.rep_base + o].kprimes;
            if (K <= 0 || K > a.kcap) continue;
            const int64_t mod_off = Q.mod_off0 + (int64_t)o * Q.nb;  // repetitions' residues follow each other
            for (int i = 0; i < K; ++i) {
                const PrimeDev &P = a.primes[i];
                const RingM R{P.p, P.pinv_neg};
                uint32_t v = lane < Q.nb ? a.modp[(size_t)i * a.mod_plane + mod_off + lane] : 0u;
                for (int off = 32; off > 0; off >>= 1) v = R.add(v, __shfl_down(v, off, 64));
                if (lane == 0) s_res[o * kMaxPrimes + i] = v;
            }
        }
    }
    __syncthreads();
    if (t < Q.d) {
        const RepDesc D = a.reps[Q.rep_base + t];
        // this repetition's record lives in registers; written back once at the end
        RepDev rp = a.rs[Q.rep_base + t];
        // additions on any term's path to a sum: its thread's serial sum (per_thread - 1),
        // block_sum (6 shuffle levels, then the kThreads / 64 wavefront sums one after
        // another) and the tree of depth 6 over the nb <= 64 block partials above
        const double per_thread = ceil(m / ((double)D.nb * kThreads));
        const double n_eff = per_thread + 6.0 + kThreads / 64 + 6.0;
        if constexpr (STAGE != 2) {
            rp.kprimes = 0;
            rp.status = 0;
            rp.window = 0;
            rp.bound = 0.0;
            if (plan == CS_PLAN_DOT) {
                unsigned __int128 s = 0;
                double fs = 0.0, fa = 0.0;
                for (int b = 0; b < D.nb; ++b) {
                    const unsigned long long *p = a.dot + (D.dot_off + b) * 4;
                    s += ((unsigned __int128)p[1] << 64) | p[0];
                    fs += __longlong_as_double((long long)p[2]);
                    fa += __longlong_as_double((long long)p[3]);
                }
                // fa sums |x_j y_j| with at most n_eff + nb additions per term (each
                // product rounded once): the true sum of |terms| is at most
                // fa (1 + (n_eff + nb + 2) u) and bounds every partial sum, so below 2^126
                // the wrapped 128-bit integer is the exact inner product
                const double bnd = fa * (1.0 + (n_eff + D.nb + 4.0) * u * 1.01);
                if (bnd < 0x1p126) {
                    const __int128 x = (__int128)s;
                    rp.lo = (int64_t)(uint64_t)s;
                    rp.hi = (int64_t)(uint64_t)(s >> 64);
                    rp.exact = 1;
                    rp.value = i128_to_double(x);
                    rp.xf = rp.value;
                } else {
                    rp.lo = rp.hi = 0;
                    rp.exact = 0;
                    rp.status = 1;
                    rp.value = fs;
                    rp.xf = fs;
                    rp.bound = bnd;
                }
            } else {
                // norms of each relation's sketch at this repetition (upper bounds)
                // per-relation values live in LDS (indexed loops over r would
                // otherwise put per-thread arrays in scratch memory)
                const double up = 1.0 + (n_eff + 4.0) * u * 1.01;
                auto s2 = [&](int k) { return s_q2[k * Q.d + t] * up; };
                auto s1 = [&](int k) { return s_l1[k * Q.d + t] * up; };
                if (plan == CS_PLAN_SPECTRAL) {
                    const double sum = s_sum[t], sabs = s_sabs[t];
                    const double *mx = s_mx + t * kMaxRel;
                    const double xf = sum / m;
                    // fp64 FFT error (radix-2 Cooley-Tukey, twiddles within 2u):
                    // ||fl(FFT z) - FFT z||_2 <= kappa sqrt(m) ||z||_2.
                    const double g4 = 4.0 * u / (1.0 - 4.0 * u);
                    const double eta = 2.0 * u + g4 * (1.41421356237309515 + 2.0 * u);
                    const double kappa = 2.0 * (Q.log2m + 3) * eta;
                    const double sm = sqrt(m) * (1.0 + 4.0 * u);
                    double *e = s_stage + t * 3 * kMaxRel;
                    double *N = e + kMaxRel;
                    double *M = N + kMaxRel;
                    const int n_sk = Q.r * Q.d;
                    for (int k = 0; k < Q.r; ++k) {
                        // packed partner: sketch index s ^ 1 within the query
                        const int sidx = k * Q.d + t;
                        double z2 = s2(k);
                        const int ps = sidx ^ 1;
                        if (ps < n_sk) z2 += s_q2[ps] * up;
                        e[k] = kappa * sm * sqrt(z2) * (1.0 + 4.0 * u);
                        N[k] = sm * sqrt(s2(k)) * (1.0 + 4.0 * u) + e[k];
                        M[k] = mx[k] * (1.0 + 4.0 * u) + e[k];
                    }
                    double dT = 0.0;
                    for (int k = 0; k < Q.r; ++k) {
                        double best = INFINITY;
                        for (int j = 0; j < Q.r; ++j) {
                            if (j == k) continue;
                            double v = N[j];
                            for (int i = 0; i < Q.r; ++i)
                                if (i != j && i != k) v *= M[i];
                            best = fmin(best, v);
                        }
                        dT += e[k] * best;
                    }
                    const double rho = ((Q.r - 1) * 3.0 + n_eff + 4.0) * u * 1.01;
                    const double bound = 2.0 * (dT + rho * sabs) / m * (1.0 + 1e-10);
                    rp.xf = xf;
                    rp.bound = bound;
                    if (bound < 0.49 && fabs(xf) + bound < 0x1p53) {
                        const __int128 x = (__int128)(int64_t)rint(xf);
                        rp.lo = (int64_t)(uint64_t)(unsigned __int128)x;
                        rp.hi = (int64_t)(uint64_t)((unsigned __int128)x >> 64);
                        rp.exact = 1;
                        rp.value = (double)rint(xf);
                    } else {
                        rp.exact = 0;
                        rp.value = xf;
                        rp.lo = rp.hi = 0;
                        if (isfinite(bound) && isfinite(xf)) {
                            // window around xf when xf fits in int128, else full centred range
                            rp.window = fabs(xf) < 0x1p120 ? 1 : 0;
                            const double need = rp.window ? log2(2.0 * bound + 4.0) + 1.0
                                                          : log2(2.0 * (fabs(xf) + bound) + 4.0) + 1.0;
                            double have = 0.0;
                            int K = 0;
                            while (K < kMaxPrimes && have <= need) have += a.crt.log2p[K++];
                            if (have > need) rp.kprimes = K;
                            else rp.status = 1;
                        } else {
                            rp.status = 1;
                        }
                    }
                } else {  // GENERAL: primes to cover 2 * prod_k ||c_k||_1 + 2
                    double lb = 0.0;
                    bool zero = false;
                    for (int k = 0; k < Q.r; ++k) {
                        if (s1(k) == 0.0) zero = true;
                        lb += log2(s1(k));
                    }
                    rp.exact = 0;
                    rp.value = 0.0;
                    rp.xf = 0.0;
                    if (zero) {
                        rp.exact = 1;
                        rp.lo = rp.hi = 0;
                    } else {
                        const double need = lb + 3.0;
                        double have = 0.0;
                        int K = 0;
                        while (K < kMaxPrimes && have <= need) have += a.crt.log2p[K++];
                        if (have > need) rp.kprimes = K;
                        else rp.status = 1;
                    }
                }
            }
        }
        if (STAGE != 1 && rp.kprimes > 0 && rp.kprimes <= a.kcap) {  // stage 2: residues -> exact value
            const int K = rp.kprimes;
            uint32_t *res = s_res + t * kMaxPrimes, *dig = s_dig + t * kMaxPrimes;
            for (int i = 0; i < K; ++i) {
                const PrimeDev &P = a.primes[i];
                const RingM R{P.p, P.pinv_neg};
                uint32_t s = res[i];  // the sum of the block partials, from above
                if (plan == CS_PLAN_SPECTRAL) s = R.mul(s, P.minv[Q.log2m]);
                res[i] = R.mul(s, 1u);  // out of Montgomery form
            }
            if (plan == CS_PLAN_SPECTRAL && rp.window) {
                const __int128 x0 = double_to_i128(rint(rp.xf));
                for (int i = 0; i < K; ++i) {
                    const uint32_t p = a.crt.p[i];
                    const uint32_t x0m = mod_i128(x0, p);
                    res[i] = (uint32_t)(((uint64_t)res[i] + p - x0m) % p);
                }
                garner(res, K, a.crt, dig);
                __int128 delta;
                double dd;
                if (digits_to_i128(dig, K, a.crt, &delta, &dd)) {
                    const __int128 x = x0 + delta;
                    rp.lo = (int64_t)(uint64_t)(unsigned __int128)x;
                    rp.hi = (int64_t)(uint64_t)((unsigned __int128)x >> 64);
                    rp.exact = 1;
                    rp.value = i128_to_double(x);
                } else {
                    rp.status = 1;
                }
            } else {
                garner(res, K, a.crt, dig);
                __int128 x;
                double dv;
                if (digits_to_i128(dig, K, a.crt, &x, &dv)) {
                    rp.lo = (int64_t)(uint64_t)(unsigned __int128)x;
                    rp.hi = (int64_t)(uint64_t)((unsigned __int128)x >> 64);
                    rp.exact = 1;
                    rp.value = i128_to_double(x);
                } else {
                    rp.exact = 0;
                    rp.value = dv;
                    rp.status = 1;
                }
            }
        }
        a.rs[Q.rep_base + t] = rp;
        if constexpr (STAGE != 2) a.kp[Q.rep_base + t] = rp.kprimes;
        s_val[t] = rp.value;
        s_ex[t] = rp.exact;
        s_lo[t] = rp.lo;
        s_hi[t] = rp.hi;
        s_kp[t] = rp.kprimes;
    }
    __syncthreads();
    if (t < Q.d) {
        // median (lower middle) by rank: total order on (fp64 value, exact flag, exact
        // integer when present, repetition index); for exact repetitions this is the
        // order of the integers, fp64 rounding being monotone
        const double v = s_val[t];
        const int ex = s_ex[t];
        const __int128 x = ex ? (__int128)(((unsigned __int128)(uint64_t)s_hi[t] << 64) | (uint64_t)s_lo[t]) : 0;
        int rank = 0, n_mod = 0;
        for (int i = 0; i < Q.d; ++i) {
            n_mod += s_kp[i] > 0;
            const double vi = s_val[i];
            bool less;
            if (vi != v) {
                less = vi < v;
            } else if (s_ex[i] != ex) {
                less = s_ex[i] < ex;
            } else {
                const __int128 xi =
                    s_ex[i] ? (__int128)(((unsigned __int128)(uint64_t)s_hi[i] << 64) | (uint64_t)s_lo[i]) : 0;
                less = xi != x ? xi < x : i < t;
            }
            rank += less;
        }
        if (rank == (Q.d - 1) / 2) {
            OutDev &o = a.outs[blockIdx.x];
            o.value = v;
            o.lo = s_lo[t];
            o.hi = s_hi[t];
            o.exact = ex;
            o.fits = ex && x >= (__int128)INT64_MIN && x <= (__int128)INT64_MAX;
            o.n_modular = n_mod;
            o.median_rep = t;
        }
    }
}

// Asynchronous results: the finalize outputs written as cs_estimate_t into memory the
// caller reads after the stream passes (device memory or pinned host memory).
__global__ void k_publish(const OutDev *__restrict__ outs, const QDesc *__restrict__ qs, int nq, cs_estimate_t *dst)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const OutDev o = outs[q];
    cs_estimate_t e;
    e.value = o.value;
    e.exact = o.exact;
    e.fits_i64 = o.fits;
    e.value_i64 = o.fits ? o.lo : 0;
    e.d = qs[q].d;
    e.n_modular = o.n_modular;
    dst[q] = e;
}

// ---------------------------------------------------------------- host: primes and tables

uint32_t host_mont_mul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv_neg)
{
    const uint64_t t = (uint64_t)a * b;
    const uint32_t q = (uint32_t)t * pinv_neg;
    const uint32_t u = (uint32_t)((t + (uint64_t)q * p) >> 32);
    return u >= p ? u - p : u;
}

uint64_t powmod(uint64_t b, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    b %= p;
    while (e) {
        if (e & 1) r = (unsigned __int128)r * b % p;
        b = (unsigned __int128)b * b % p;
        e >>= 1;
    }
    return r;
}

bool is_prime_u32(uint64_t n)
{
    if (n < 2) return false;
    for (uint64_t q : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull})
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : {2ull, 7ull, 61ull}) {  // deterministic below 2^32
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s; ++i) {
            x = (unsigned __int128)x * x % n;
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

std::vector<PrimeInfo> build_primes()
{
    std::vector<PrimeInfo> out;
    const uint64_t step = 1ull << kMaxLog2N;
    for (uint64_t c = ((1ull << 31) - 1) / step; c > 0 && (int)out.size() < kMaxPrimes; --c) {
        const uint64_t p = c * step + 1;
        if (p >= (1ull << 31) || !is_prime_u32(p)) continue;
        PrimeInfo P{};
        P.p = (uint32_t)p;
        uint32_t inv = 1;  // Newton iteration for p^-1 mod 2^32
        for (int i = 0; i < 5; ++i) inv *= 2u - (uint32_t)p * inv;
        P.pinv_neg = (uint32_t)(0u - inv);
        P.r2 = (uint32_t)(((unsigned __int128)1 << 64) % p);
        P.r3 = (uint32_t)((unsigned __int128)P.r2 * ((1ull << 32) % p) % p);
        const uint64_t m64 = P.r2;  // 2^64 mod p
        const uint64_t neg = (p - m64) % p;
        P.neg2_64 = (uint32_t)((unsigned __int128)neg * ((1ull << 32) % p) % p);
        // generator: p - 1 = c * 2^21
        std::vector<uint64_t> fs{2};
        uint64_t cc = c;
        for (uint64_t q = 2; q * q <= cc; ++q)
            if (cc % q == 0) {
                if (q != 2) fs.push_back(q);
                while (cc % q == 0) cc /= q;
            }
        if (cc > 1 && cc != 2) fs.push_back(cc);
        uint64_t g = 2;
        for (;; ++g) {
            bool ok = true;
            for (uint64_t q : fs)
                if (powmod(g, (p - 1) / q, p) == 1) ok = false;
            if (ok) break;
        }
        P.g = (uint32_t)g;
        out.push_back(P);
    }
    return out;
}

struct DeviceTables {
    PrimeDev *primes = nullptr;
    std::map<int, double2 *> tw;       // log2m -> twiddles
    std::map<int, uint32_t *> roots;   // log2m -> [K][2][m]
};
std::mutex g_tab_mu;
std::map<int, DeviceTables> g_tabs;

CrtTables g_crt;
bool g_crt_ready = false;

void build_crt_tables()
{
    const auto &P = ntt_primes();
    std::memset(&g_crt, 0, sizeof(g_crt));
    for (int i = 0; i < kMaxPrimes; ++i) {
        g_crt.p[i] = P[i].p;
        g_crt.log2p[i] = std::log2((double)P[i].p);
    }
    for (int j = 0; j < kMaxPrimes; ++j)
        for (int i = 0; i < kMaxPrimes; ++i)
            if (i != j) g_crt.inv[j][i] = (uint32_t)powmod(P[j].p % P[i].p, P[i].p - 2, P[i].p);
    // digits of (P_K - 1)/2 for every K: its residue mod p_i is (p_i - 1)/2
    for (int K = 1; K <= kMaxPrimes; ++K) {
        uint32_t res[kMaxPrimes];
        for (int i = 0; i < K; ++i) res[i] = (P[i].p - 1) / 2;
        for (int i = 0; i < K; ++i) {
            uint64_t x = res[i];
            for (int j = 0; j < i; ++j) {
                x = (x + P[i].p - g_crt.half[K - 1][j] % P[i].p) % P[i].p;
                x = x * g_crt.inv[j][i] % P[i].p;
            }
            g_crt.half[K - 1][i] = (uint32_t)x;
        }
    }
    g_crt_ready = true;
}

cs_status device_primes(int device, hipStream_t s, PrimeDev **out)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    DeviceTables &T = g_tabs[device];
    if (!T.primes) {
        const auto &P = ntt_primes();
        std::vector<PrimeDev> h(kMaxPrimes);
        for (int i = 0; i < kMaxPrimes; ++i) {
            PrimeDev &D = h[i];
            D.p = P[i].p;
            D.pinv_neg = P[i].pinv_neg;
            D.r2 = P[i].r2;
            D.r3 = P[i].r3;
            D.neg2_64 = P[i].neg2_64;
            D.one = (uint32_t)((1ull << 32) % P[i].p);
            for (int L = 0; L <= kMaxLog2N; ++L) {
                const uint64_t inv_m = powmod(powmod(2, L, P[i].p), P[i].p - 2, P[i].p);
                D.minv[L] = (uint32_t)((unsigned __int128)inv_m * ((1ull << 32) % P[i].p) % P[i].p);
            }
        }
        PrimeDev *dp = nullptr;
        if (hipMalloc(&dp, sizeof(PrimeDev) * kMaxPrimes) != hipSuccess)
            return fail(CS_ENOMEM, "prime table allocation failed");
        CSK_HIP(hipMemcpy(dp, h.data(), sizeof(PrimeDev) * kMaxPrimes, hipMemcpyHostToDevice));
        T.primes = dp;
    }
    if (!g_crt_ready) build_crt_tables();
    *out = T.primes;
    (void)s;
    return CS_OK;
}

}  // namespace

const std::vector<PrimeInfo> &ntt_primes()
{
    static const std::vector<PrimeInfo> P = build_primes();
    return P;
}

// The table builders compute on the host and upload outside the table lock (a thread
// that needs a table never waits on the lock while another thread's allocation or copy
// is in flight); when two threads build the same table at once, the first insert wins and
// the other frees its copy.
const double *twiddles_f64(int device, int log2m, hipStream_t s, cs_status *st)
{
    {
        std::lock_guard<std::mutex> lk(g_tab_mu);
        DeviceTables &T = g_tabs[device];
        auto it = T.tw.find(log2m);
        if (it != T.tw.end()) {
            *st = CS_OK;
            return reinterpret_cast<const double *>(it->second);
        }
    }
    const size_t m = (size_t)1 << log2m;
    std::vector<double2> h(m);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    // w^k = (cos, -sin)(2 pi k / m): the long-double cosine and sine are evaluated on the
    // first octant only and the rest follows by the exact symmetries
    // (c, s)(pi/2 - x) = (s, c), (c, s)(pi/2 + x) = (-s, c), (c, s)(pi + x) = (-c, -s)
    auto cs = [&](size_t k) -> std::pair<double, double> {  // (cos, sin)(2 pi k / m), k <= m / 8
        const long double a = two_pi * (long double)k / (long double)m;
        return {(double)cosl(a), (double)sinl(a)};
    };
    auto trig = [&](size_t k) -> std::pair<double, double> {
        if (m < 8) return cs(k);
        const size_t q = m / 4, o = m / 8;
        bool neg = false;
        if (k >= 2 * q) {  // pi + x
            k -= 2 * q;
            neg = true;
        }
        std::pair<double, double> v;
        if (k <= o) {
            v = cs(k);
        } else if (k <= q) {  // pi/2 - x, x = 2 pi (q - k) / m
            const auto t = cs(q - k);
            v = {t.second, t.first};
        } else if (k <= q + o) {  // pi/2 + x, x = 2 pi (k - q) / m
            const auto t = cs(k - q);
            v = {-t.second, t.first};
        } else {  // pi - x, x = 2 pi (2q - k) / m: (c, s)(pi - x) = (-c, s)
            const auto t = cs(2 * q - k);
            v = {-t.first, t.second};
        }
        if (neg) v = {-v.first, -v.second};
        return v;
    };
    for (size_t k = 0; k < m; ++k) {
        const auto v = trig(k);
        h[k] = make_double2(v.first, -v.second);
    }
    double2 *dp = nullptr;
    if (hipMalloc(&dp, m * sizeof(double2)) != hipSuccess) {
        *st = fail(CS_ENOMEM, "twiddle table allocation failed");
        return nullptr;
    }
    if (hipMemcpy(dp, h.data(), m * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dp);
        *st = fail(CS_EDEVICE, "twiddle upload failed");
        return nullptr;
    }
    (void)s;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    DeviceTables &T = g_tabs[device];
    auto ins = T.tw.emplace(log2m, dp);
    if (!ins.second) (void)hipFree(dp);  // built meanwhile by another thread
    *st = CS_OK;
    return reinterpret_cast<const double *>(ins.first->second);
}

const uint32_t *roots_mod(int device, int log2m, int /*prime*/, bool /*inverse*/, hipStream_t s, cs_status *st)
{
    {
        std::lock_guard<std::mutex> lk(g_tab_mu);
        DeviceTables &T = g_tabs[device];
        auto it = T.roots.find(log2m);
        if (it != T.roots.end()) {
            *st = CS_OK;
            return it->second;
        }
    }
    const auto &P = ntt_primes();
    const size_t m = (size_t)1 << log2m;
    std::vector<uint32_t> h((size_t)kMaxPrimes * 2 * m);
    for (int i = 0; i < kMaxPrimes; ++i) {
        const uint64_t p = P[i].p;
        const uint64_t w = powmod(P[i].g, (p - 1) >> log2m, p);
        const uint64_t wi = powmod(w, p - 2, p);
        // p < 2^31: products of two residues fit 64 bits; the table holds the Montgomery
        // forms w^k 2^32 mod p, stepped directly
        const uint64_t R = (1ull << 32) % p;
        for (int dir = 0; dir < 2; ++dir) {
            uint64_t acc = R;  // Montgomery form of w^0
            const uint64_t step = dir ? wi : w;
            uint32_t *dst = h.data() + ((size_t)(2 * i + dir) << log2m);
            for (size_t k = 0; k < m; ++k) {
                dst[k] = (uint32_t)acc;
                acc = acc * step % p;
            }
        }
    }
    uint32_t *dp = nullptr;
    if (hipMalloc(&dp, h.size() * sizeof(uint32_t)) != hipSuccess) {
        *st = fail(CS_ENOMEM, "root table allocation failed");
        return nullptr;
    }
    if (hipMemcpy(dp, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dp);
        *st = fail(CS_EDEVICE, "root table upload failed");
        return nullptr;
    }
    (void)s;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    DeviceTables &T = g_tabs[device];
    auto ins = T.roots.emplace(log2m, dp);
    if (!ins.second) (void)hipFree(dp);  // built meanwhile by another thread
    *st = CS_OK;
    return ins.first->second;
}

// ---------------------------------------------------------------- host: batched estimate engine

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Waits for the stream by polling: the results are a few kilobytes, due within
// microseconds of the last kernel, and a blocking wait's wake-up costs more than that.
cs_status wait_results(hipStream_t s)
{
    for (;;) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) return CS_OK;
        if (e != hipErrorNotReady) return fail(CS_EDEVICE, std::string("hipStreamQuery: ") + hipGetErrorString(e));
    }
}

int ceil_log2(uint32_t x)
{
    int L = 0;
    while ((1ull << L) < x) ++L;
    return L;
}

int nblocks_for(uint32_t m)
{
    // two elements per thread: enough workgroups to fill the chip for small batches;
    // at most 64, one partial per lane of the wavefront that reduces them (k_finalize)
    size_t nb = (size_t)m / (kThreads * 2);
    if (nb < 1) nb = 1;
    if (nb > 64) nb = 64;
    return (int)nb;
}

// Workspace growth by at least half the current size, so that batches of varying size
// (the serving loop's) reallocate a logarithmic number of times.
size_t grown(size_t have, size_t need) { return std::max(need, have + have / 2); }

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    }
};

}  // namespace

cs_status estimate_batch(Handle *const *hs, int nq, hipStream_t s, cs_estimate_t *outs, const cs_reps_t *reps_out,
                         EstimateWork &ws, cs_estimate_t *async_out)
{
    if (nq <= 0) return CS_OK;
    const int device = hs[0]->device;
    // one split per transform length for the whole estimate (the tuning table may change
    // between estimates, never inside one)
    std::map<int, int> split_cache;
    auto split_of = [&](int L) {
        auto it = split_cache.find(L);
        if (it != split_cache.end()) return it->second;
        const int S = split_for(device, L);
        split_cache.emplace(L, S);
        return S;
    };
    for (int q = 0; q < nq; ++q)
        if (hs[q]->device != device) return fail(CS_EINVAL, "batched estimate: handles on different devices");
    PrimeDev *primes = nullptr;
    cs_status st = device_primes(device, s, &primes);
    if (st != CS_OK) return st;

    // ---- host tables
    std::vector<QDesc> qd(nq);
    std::vector<RepDesc> rd;
    std::vector<SkDesc> sd;
    std::vector<int32_t> dot_idx;
    struct Group {
        int log2m, S;
        std::vector<int> queries;
        std::vector<int32_t> rep_idx;
        std::vector<const int64_t *> re, im;
        std::vector<const int64_t *> mod_ptrs;  // every sketch, (query, relation, repetition) order
        std::vector<int32_t> rep_of;            // repetition of each of those sketches
        size_t z_off = 0;
    };
    std::map<int, Group> groups;
    std::vector<int> general_q;
    int64_t norm_off = 0, spec_off = 0, dot_off = 0, mod_off = 0;
    for (int q = 0; q < nq; ++q) {
        const Handle &h = *hs[q];
        const int r = h.g.n_rel, d = (int)h.d, L = h.log2m;
        const int nb = nblocks_for(h.m);
        QDesc &Q = qd[q];
        Q.plan = h.g.plan;
        Q.r = r;
        Q.d = d;
        Q.log2m = L;
        Q.m = h.m;
        Q.rep_base = (int32_t)rd.size();
        Q.nb = nb;
        Q.norm_off0 = norm_off;
        Q.spec_off0 = spec_off;
        Q.mod_off0 = mod_off;
        const int sk_base = (int)sd.size();
        const size_t m = h.m;
        if (Q.plan != CS_PLAN_DOT) {
            for (int k = 0; k < r; ++k)
                for (int t = 0; t < d; ++t) {
                    SkDesc S;
                    S.p = rel_counters(h, k) + (size_t)t * m;
                    S.log2m = L;
                    S.m = h.m;
                    S.nb = nb;
                    S.off = norm_off;
                    norm_off += nb;
                    sd.push_back(S);
                }
        }
        int vec_base = 0, mod_base = 0;
        Group *G = nullptr;
        if (Q.plan == CS_PLAN_SPECTRAL) {
            G = &groups[L];
            G->log2m = L;
            G->S = split_of(L);
            G->queries.push_back(q);
            vec_base = (int)G->re.size();
            const int n_sk = r * d;
            for (int v = 0; v < (n_sk + 1) / 2; ++v) {
                const int s0 = 2 * v, s1 = 2 * v + 1;
                G->re.push_back(sd[sk_base + s0].p);
                G->im.push_back(s1 < n_sk ? sd[sk_base + s1].p : nullptr);
            }
            mod_base = (int)G->mod_ptrs.size();
            for (int j = 0; j < n_sk; ++j) {
                G->mod_ptrs.push_back(sd[sk_base + j].p);
                G->rep_of.push_back(Q.rep_base + j % d);
            }
        }
        if (Q.plan == CS_PLAN_GENERAL) general_q.push_back(q);
        for (int t = 0; t < d; ++t) {
            RepDesc D{};
            D.c0 = rel_counters(h, 0) + (size_t)t * m;
            D.c1 = rel_counters(h, 1) + (size_t)t * m;
            D.q = q;
            D.t = t;
            D.log2m = L;
            D.S = split_of(L);
            D.m = h.m;
            D.r = r;
            D.d = d;
            D.conj = h.g.conj_mask;
            D.vec_base = vec_base;
            D.nb = nb;
            D.sk_base = sk_base;
            D.mod_vec_base = mod_base;
            D.spec_off = spec_off;
            D.dot_off = dot_off;
            D.mod_off = mod_off;
            mod_off += nb;
            if (Q.plan == CS_PLAN_SPECTRAL) {
                spec_off += (int64_t)nb * (2 + r);
                G->rep_idx.push_back((int32_t)rd.size());
            }
            if (Q.plan == CS_PLAN_DOT) {
                dot_off += nb;
                dot_idx.push_back((int32_t)rd.size());
            }
            rd.push_back(D);
        }
    }
    const int n_rep = (int)rd.size();
    const int64_t mod_plane = mod_off;
    if (async_out && !general_q.empty())
        return fail(CS_EINVAL, "asynchronous estimates need queries without the general plan");

    // ---- workspace layout
    Carve c;
    const size_t o_q = c.take(qd.size() * sizeof(QDesc));
    const size_t o_rep = c.take(rd.size() * sizeof(RepDesc));
    const size_t o_sk = c.take(std::max<size_t>(1, sd.size()) * sizeof(SkDesc));
    const size_t o_dotidx = c.take(std::max<size_t>(1, dot_idx.size()) * sizeof(int32_t));
    // block prefixes of the flattened launches
    std::vector<int64_t> sk_pre(sd.size() + 1, 0), dot_pre(dot_idx.size() + 1, 0);
    for (size_t i = 0; i < sd.size(); ++i) sk_pre[i + 1] = sk_pre[i] + sd[i].nb;
    for (size_t i = 0; i < dot_idx.size(); ++i) dot_pre[i + 1] = dot_pre[i] + rd[dot_idx[i]].nb;
    const size_t o_skpre = c.take(sk_pre.size() * sizeof(int64_t));
    const size_t o_dotpre = c.take(dot_pre.size() * sizeof(int64_t));
    std::vector<size_t> o_gidx, o_gre, o_gim, o_gpre, o_gptr, o_grepof;
    std::vector<std::vector<int64_t>> g_pre;
    size_t z_total = 0;
    for (auto &kv : groups) {
        Group &G = kv.second;
        o_gidx.push_back(c.take(G.rep_idx.size() * sizeof(int32_t)));
        std::vector<int64_t> pre(G.rep_idx.size() + 1, 0);
        for (size_t i = 0; i < G.rep_idx.size(); ++i) pre[i + 1] = pre[i] + rd[G.rep_idx[i]].nb;
        o_gpre.push_back(c.take(pre.size() * sizeof(int64_t)));
        g_pre.push_back(std::move(pre));
        o_gre.push_back(c.take(G.re.size() * sizeof(void *)));
        o_gim.push_back(c.take(G.im.size() * sizeof(void *)));
        o_gptr.push_back(c.take(G.mod_ptrs.size() * sizeof(void *)));
        o_grepof.push_back(c.take(G.rep_of.size() * sizeof(int32_t)));
        G.z_off = z_total;
        z_total += align_up(G.re.size() * ((size_t)1 << G.log2m) * sizeof(double2));
    }
    const size_t host_tables = c.off;
    const size_t o_norms = c.take(std::max<int64_t>(1, norm_off) * 2 * sizeof(double));
    const size_t o_spec = c.take(std::max<int64_t>(1, spec_off) * sizeof(double));
    const size_t o_dot = c.take(std::max<int64_t>(1, dot_off) * 4 * sizeof(unsigned long long));
    const size_t o_modp = c.take((size_t)kMaxPrimes * std::max<int64_t>(1, mod_plane) * sizeof(uint32_t));
    const size_t o_rs = c.take((size_t)n_rep * sizeof(RepDev));  // [records | outputs]: one download
    const size_t o_outs = c.take((size_t)nq * sizeof(OutDev));
    const size_t o_kp = c.take((size_t)n_rep * sizeof(int32_t));
    const size_t o_Z = c.take(z_total);
    if (ws.bytes < c.off) {
        if (ws.buf) {
            CSK_HIP(hipStreamSynchronize(s));
            hipFree(ws.buf);
        }
        const size_t want = grown(ws.bytes, c.off);
        ws.buf = nullptr;
        ws.bytes = 0;
        if (hipMalloc(&ws.buf, want) != hipSuccess) return fail(CS_ENOMEM, "estimate workspace");
        ws.bytes = want;
    }
    char *wb = static_cast<char *>(ws.buf);
    // pinned host staging: [tables | repetition records | outputs | modular-step tables]
    Carve hc;
    const size_t h_img = hc.take(host_tables);
    const size_t h_rs = hc.take((size_t)n_rep * sizeof(RepDev));  // same relative layout as the device's
    const size_t h_outs = hc.take((size_t)nq * sizeof(OutDev));
    const size_t h_mod = hc.take(align_up(sd.size() * sizeof(void *)) + align_up((size_t)n_rep * sizeof(int32_t)) +
                                 (size_t)(n_rep + 1 + (int)groups.size()) * sizeof(int64_t) +
                                 3 * 256 * (groups.size() + 1));
    // an asynchronous estimate may still be uploading from the staging area
    if (ws.upload_pending) {
        CSK_HIP(hipEventSynchronize(ws.ev_upload));
        ws.upload_pending = false;
    }
    if (ws.host_bytes < hc.off) {
        const size_t want = grown(ws.host_bytes, hc.off);
        if (ws.host) hipHostFree(ws.host);
        ws.host = nullptr;
        ws.host_bytes = 0;
        if (hipHostMalloc(&ws.host, want, hipHostMallocDefault) != hipSuccess)
            return fail(CS_ENOMEM, "estimate host staging");
        ws.host_bytes = want;
    }
    char *hb = static_cast<char *>(ws.host);
    RepDev *hr = reinterpret_cast<RepDev *>(hb + h_rs);
    OutDev *ho = reinterpret_cast<OutDev *>(hb + h_outs);
    // host image of the tables, one upload
    struct HostImg {
        char *p;
        size_t n;
        char *data() { return p; }
        size_t size() const { return n; }
    } img{hb + h_img, host_tables};
    std::memset(img.data(), 0, img.size());
    std::memcpy(img.data() + o_q, qd.data(), qd.size() * sizeof(QDesc));
    std::memcpy(img.data() + o_rep, rd.data(), rd.size() * sizeof(RepDesc));
    if (!sd.empty()) std::memcpy(img.data() + o_sk, sd.data(), sd.size() * sizeof(SkDesc));
    if (!dot_idx.empty()) std::memcpy(img.data() + o_dotidx, dot_idx.data(), dot_idx.size() * sizeof(int32_t));
    std::memcpy(img.data() + o_skpre, sk_pre.data(), sk_pre.size() * sizeof(int64_t));
    std::memcpy(img.data() + o_dotpre, dot_pre.data(), dot_pre.size() * sizeof(int64_t));
    {
        int gi = 0;
        for (auto &kv : groups) {
            Group &G = kv.second;
            std::memcpy(img.data() + o_gidx[gi], G.rep_idx.data(), G.rep_idx.size() * sizeof(int32_t));
            std::memcpy(img.data() + o_gpre[gi], g_pre[gi].data(), g_pre[gi].size() * sizeof(int64_t));
            std::memcpy(img.data() + o_gre[gi], G.re.data(), G.re.size() * sizeof(void *));
            std::memcpy(img.data() + o_gim[gi], G.im.data(), G.im.size() * sizeof(void *));
            std::memcpy(img.data() + o_gptr[gi], G.mod_ptrs.data(), G.mod_ptrs.size() * sizeof(void *));
            std::memcpy(img.data() + o_grepof[gi], G.rep_of.data(), G.rep_of.size() * sizeof(int32_t));
            ++gi;
        }
    }
    CSK_HIP(hipMemcpyAsync(wb, img.data(), img.size(), hipMemcpyHostToDevice, s));
    if (async_out) {
        if (!ws.ev_upload) CSK_HIP(hipEventCreateWithFlags(&ws.ev_upload, hipEventDisableTiming));
        CSK_HIP(hipEventRecord(ws.ev_upload, s));
        ws.upload_pending = true;
    }
    const QDesc *d_q = reinterpret_cast<const QDesc *>(wb + o_q);
    RepDesc *d_rep = reinterpret_cast<RepDesc *>(wb + o_rep);
    const SkDesc *d_sk = reinterpret_cast<const SkDesc *>(wb + o_sk);
    double *d_norms = reinterpret_cast<double *>(wb + o_norms);
    double *d_spec = reinterpret_cast<double *>(wb + o_spec);
    unsigned long long *d_dot = reinterpret_cast<unsigned long long *>(wb + o_dot);
    uint32_t *d_modp = reinterpret_cast<uint32_t *>(wb + o_modp);
    RepDev *d_rs = reinterpret_cast<RepDev *>(wb + o_rs);
    int32_t *d_kp = reinterpret_cast<int32_t *>(wb + o_kp);
    OutDev *d_outs = reinterpret_cast<OutDev *>(wb + o_outs);

    // ---- speculative modular step: when no query has a general plan and the workspace
    // is modest, the residues of the first ks primes are computed for every repetition
    // beside the fp64 pass, and one finalize launch uses both (no round trip to the
    // host); ks is what the previous estimate on this workspace needed (kSpecPrimes for
    // the first).  A repetition that needs more primes takes the stage below.  The two
    // chains share nothing until the finalize: with at most kOverlapPrimes primes and at
    // least kOverlapMinResidues residues the modular one runs on the workspace's side
    // stream (forked behind the table upload, joined before the finalize), so that the
    // launches of either overlap the other's.  Measured: overlapping five primes at
    // m = 2^18 with 75 sketch vectors made the estimate 10% slower (the modular chain
    // fills the chip alone), two or three primes 1-13% faster; for small estimates
    // (thousands of handles with m <= 2^16, one estimate each) the fork and join cost
    // more than they save and halved the estimates per second.
    int kdone = 0;
    const int ks = ws.spec_k >= 0 ? std::min(ws.spec_k, kSpecPrimes) : kSpecPrimes;
    bool spec = false, overlap = false;
    hipStream_t ms = s;  // stream of the speculative modular chain
    if (ks > 0 && general_q.empty() && !groups.empty()) {
        size_t spec_bytes = 0;
        for (auto &kv : groups)
            spec_bytes += align_up((size_t)ks * kv.second.mod_ptrs.size() * ((size_t)1 << kv.second.log2m) *
                                   sizeof(uint32_t));
        if (spec_bytes <= kSpecBudget) {
            overlap = ks <= kOverlapPrimes && spec_bytes / sizeof(uint32_t) >= kOverlapMinResidues;
            if (overlap && !ws.side) {
                CSK_HIP(hipStreamCreateWithFlags(&ws.side, hipStreamNonBlocking));
                CSK_HIP(hipEventCreateWithFlags(&ws.ev_fork, hipEventDisableTiming));
                CSK_HIP(hipEventCreateWithFlags(&ws.ev_join, hipEventDisableTiming));
            }
            if (ws.mod_bytes < spec_bytes) {
                CSK_HIP(hipStreamSynchronize(s));
                if (ws.side) CSK_HIP(hipStreamSynchronize(ws.side));
                const size_t want = grown(ws.mod_bytes, spec_bytes);
                if (ws.mod) hipFree(ws.mod);
                ws.mod = nullptr;
                ws.mod_bytes = 0;
                if (hipMalloc(&ws.mod, want) != hipSuccess) return fail(CS_ENOMEM, "modular workspace");
                ws.mod_bytes = want;
            }
            std::vector<const uint32_t *> groots;
            for (auto &kv : groups) {  // tables first: built and uploaded synchronously
                groots.push_back(roots_mod(device, kv.second.log2m, 0, false, s, &st));
                if (!groots.back()) return st;
            }
            spec = true;
            if (overlap) {
                ms = ws.side;
                CSK_HIP(hipEventRecord(ws.ev_fork, s));
                CSK_HIP(hipStreamWaitEvent(ws.side, ws.ev_fork, 0));
            }
            char *mod_cur = static_cast<char *>(ws.mod);
            int gi = 0;
            for (auto &kv : groups) {
                Group &G = kv.second;
                const int vpp = (int)G.mod_ptrs.size();
                uint32_t *N = reinterpret_cast<uint32_t *>(mod_cur);
                mod_cur += align_up((size_t)ks * vpp * ((size_t)1 << G.log2m) * sizeof(uint32_t));
                st = ntt_forward(reinterpret_cast<const int64_t *const *>(wb + o_gptr[gi]), vpp, ks, N, G.log2m,
                                 G.S, primes, groots[gi], G.log2m, ms);
                if (st != CS_OK) return st;
                hipLaunchKernelGGL(k_spec_mod, dim3((unsigned)g_pre[gi].back(), ks), dim3(kThreads), 0, ms, N,
                                   vpp, d_rep, reinterpret_cast<const int32_t *>(wb + o_gidx[gi]),
                                   reinterpret_cast<const int64_t *>(wb + o_gpre[gi]), (int)G.rep_idx.size(),
                                   primes, mod_plane, d_modp, nullptr);
                CSK_HIP(hipGetLastError());
                ++gi;
            }
            if (overlap) CSK_HIP(hipEventRecord(ws.ev_join, ws.side));
        }
    }

    // ---- stage 1
    if (!sd.empty()) {
        hipLaunchKernelGGL(k_norms, dim3((unsigned)sk_pre.back()), dim3(kThreads), 0, s, d_sk,
                           reinterpret_cast<const int64_t *>(wb + o_skpre), (int)sd.size(), d_norms);
        CSK_HIP(hipGetLastError());
    }
    if (!dot_idx.empty()) {
        hipLaunchKernelGGL(k_dot, dim3((unsigned)dot_pre.back()), dim3(kThreads), 0, s, d_rep,
                           reinterpret_cast<const int32_t *>(wb + o_dotidx),
                           reinterpret_cast<const int64_t *>(wb + o_dotpre), (int)dot_idx.size(), d_dot);
        CSK_HIP(hipGetLastError());
    }
    {
        int gi = 0;
        for (auto &kv : groups) {
            Group &G = kv.second;
            const double *tw = twiddles_f64(device, G.log2m, s, &st);
            if (!tw) return st;
            double2 *Z = reinterpret_cast<double2 *>(wb + o_Z + G.z_off);
            st = fft_f64_forward(reinterpret_cast<const int64_t *const *>(wb + o_gre[gi]),
                                 reinterpret_cast<const int64_t *const *>(wb + o_gim[gi]), (int)G.re.size(), Z,
                                 G.log2m, G.S, reinterpret_cast<const double2 *>(tw), G.log2m, s);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_spec_f64, dim3((unsigned)g_pre[gi].back()), dim3(kThreads), 0, s, Z, d_rep,
                               reinterpret_cast<const int32_t *>(wb + o_gidx[gi]),
                               reinterpret_cast<const int64_t *>(wb + o_gpre[gi]), (int)G.rep_idx.size(), d_spec);
            CSK_HIP(hipGetLastError());
            ++gi;
        }
    }
    if (overlap) CSK_HIP(hipStreamWaitEvent(s, ws.ev_join, 0));  // the modular chain joins here
    FinalizeArgs fa{};
    fa.qs = d_q;
    fa.reps = d_rep;
    fa.sks = d_sk;
    fa.norms = d_norms;
    fa.spec = d_spec;
    fa.dot = d_dot;
    fa.modp = d_modp;
    fa.mod_plane = mod_plane;
    fa.primes = primes;
    fa.crt = g_crt;
    fa.rs = d_rs;
    fa.outs = d_outs;
    fa.kp = d_kp;
    fa.kcap = kMaxPrimes;
    if (spec) {
        // both finalize stages in one launch
        fa.stage = 3;
        fa.kcap = ks;
        if (nq <= 256) hipLaunchKernelGGL((k_finalize<3, kFinThreadsFew>), dim3(nq), dim3(kFinThreadsFew), 0, s, fa);
        else hipLaunchKernelGGL((k_finalize<3, kFinThreadsMany>), dim3(nq), dim3(kFinThreadsMany), 0, s, fa);
        CSK_HIP(hipGetLastError());
        kdone = ks;
    } else {
        fa.stage = 1;
        if (nq <= 256) hipLaunchKernelGGL((k_finalize<1, kFinThreadsFew>), dim3(nq), dim3(kFinThreadsFew), 0, s, fa);
        else hipLaunchKernelGGL((k_finalize<1, kFinThreadsMany>), dim3(nq), dim3(kFinThreadsMany), 0, s, fa);
        CSK_HIP(hipGetLastError());
    }
    if (async_out) {
        // no host round trip: repetitions that need more primes than the speculative
        // step computed keep their fp64 value and exact = 0
        hipLaunchKernelGGL(k_publish, dim3((nq + 63) / 64), dim3(64), 0, s, d_outs, d_q, nq, async_out);
        CSK_HIP(hipGetLastError());
        return CS_OK;
    }
    CSK_HIP(hipMemcpyAsync(hr, d_rs, (o_outs - o_rs) + nq * sizeof(OutDev), hipMemcpyDeviceToHost, s));
    st = wait_results(s);
    if (st != CS_OK) return st;
    {
        int kmax = 0;
        for (int i = 0; i < n_rep; ++i) kmax = std::max(kmax, (int)hr[i].kprimes);
        ws.spec_k = kmax;
    }

    // ---- stage 2: modular residues for the repetitions still waiting for them
    bool any = false;
    for (int i = 0; i < n_rep; ++i) any = any || hr[i].kprimes > kdone;
    if (any) {
        // device workspace of the whole step, sized first (grows, never shrinks)
        size_t mod_need = 0;
        for (auto &kv : groups) {
            const Group &G = kv.second;
            int K = 0, vpp = 0, nidx = 0;
            for (int q : G.queries) {
                int kq = 0;
                for (int t = 0; t < qd[q].d; ++t) kq = std::max(kq, hr[qd[q].rep_base + t].kprimes);
                if (kq > kdone) {
                    K = std::max(K, kq);
                    vpp += qd[q].r * qd[q].d;
                    nidx += qd[q].d;
                }
            }
            if (K == 0) continue;
            const size_t tabs = align_up((size_t)vpp * sizeof(void *)) + align_up((size_t)nidx * sizeof(int32_t)) +
                                align_up((size_t)(nidx + 1) * sizeof(int64_t));
            mod_need += tabs + align_up((size_t)K * vpp * ((size_t)1 << G.log2m) * sizeof(uint32_t));
        }
        for (int q : general_q) {
            int K = 0;
            for (int t = 0; t < qd[q].d; ++t) K = std::max(K, hr[qd[q].rep_base + t].kprimes);
            if (K <= kdone) continue;
            mod_need += align_up((size_t)hs[q]->g.n_regs * K * qd[q].d * hs[q]->m * sizeof(uint32_t));
            if (!hs[q]->pow2)
                mod_need += 2 * align_up((size_t)K * qd[q].d * ((size_t)1 << ceil_log2(2 * hs[q]->m - 1)) *
                                         sizeof(uint32_t));
        }
        if (ws.mod_bytes < mod_need) {
            const size_t want = grown(ws.mod_bytes, mod_need);
            CSK_HIP(hipStreamSynchronize(s));
            if (ws.mod) hipFree(ws.mod);
            ws.mod = nullptr;
            ws.mod_bytes = 0;
            if (hipMalloc(&ws.mod, want) != hipSuccess) return fail(CS_ENOMEM, "modular workspace");
            ws.mod_bytes = want;
        }
        char *mod_cur = static_cast<char *>(ws.mod);
        char *mod_host = hb + h_mod;
        // spectral groups: every repetition of a query that needs one is recomputed
        for (auto &kv : groups) {
            Group &G = kv.second;
            int K = 0;
            std::vector<int> needq;
            for (int q : G.queries) {
                int kq = 0;
                for (int t = 0; t < qd[q].d; ++t) kq = std::max(kq, hr[qd[q].rep_base + t].kprimes);
                if (kq > kdone) {
                    needq.push_back(q);
                    K = std::max(K, kq);
                }
            }
            if (needq.empty()) continue;
            const uint32_t *roots = roots_mod(device, G.log2m, 0, false, s, &st);
            if (!roots) return st;
            std::vector<const int64_t *> ptrs;
            std::vector<int32_t> idx;
            for (int q : needq) {
                const int base = (int)ptrs.size();
                for (int k = 0; k < qd[q].r; ++k)
                    for (int t = 0; t < qd[q].d; ++t) ptrs.push_back(rel_counters(*hs[q], k) + (size_t)t * hs[q]->m);
                for (int t = 0; t < qd[q].d; ++t) {
                    rd[qd[q].rep_base + t].mod_vec_base = base;
                    idx.push_back(qd[q].rep_base + t);
                }
            }
            const int vpp = (int)ptrs.size();
            const size_t m = (size_t)1 << G.log2m;
            std::vector<int64_t> mpre(idx.size() + 1, 0);
            for (size_t i = 0; i < idx.size(); ++i) mpre[i + 1] = mpre[i] + rd[idx[i]].nb;
            const size_t o_mpre = align_up(ptrs.size() * sizeof(void *)) + align_up(idx.size() * sizeof(int32_t));
            const size_t tab_bytes = o_mpre + align_up(mpre.size() * sizeof(int64_t));
            char *mbc = mod_cur;
            mod_cur += tab_bytes + align_up((size_t)K * vpp * m * sizeof(uint32_t));
            char *mimg = mod_host;  // pinned; stays untouched until the call returns
            mod_host += tab_bytes;
            std::memcpy(mimg, ptrs.data(), ptrs.size() * sizeof(void *));
            std::memcpy(mimg + align_up(ptrs.size() * sizeof(void *)), idx.data(), idx.size() * sizeof(int32_t));
            std::memcpy(mimg + o_mpre, mpre.data(), mpre.size() * sizeof(int64_t));
            CSK_HIP(hipMemcpyAsync(mbc, mimg, tab_bytes, hipMemcpyHostToDevice, s));
            // updated mod_vec_base of these repetitions
            for (int q : needq)
                CSK_HIP(hipMemcpyAsync(d_rep + qd[q].rep_base, rd.data() + qd[q].rep_base, qd[q].d * sizeof(RepDesc),
                                       hipMemcpyHostToDevice, s));
            uint32_t *N = reinterpret_cast<uint32_t *>(mbc + tab_bytes);
            st = ntt_forward(reinterpret_cast<const int64_t *const *>(mbc), vpp, K, N, G.log2m, G.S, primes, roots,
                             G.log2m, s);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_spec_mod, dim3((unsigned)mpre.back(), K), dim3(kThreads), 0, s, N, vpp, d_rep,
                               reinterpret_cast<const int32_t *>(mbc + align_up(ptrs.size() * sizeof(void *))),
                               reinterpret_cast<const int64_t *>(mbc + o_mpre), (int)idx.size(), primes,
                               mod_plane, d_modp, nullptr);
            CSK_HIP(hipGetLastError());
        }
        // general plans: Alg. 3's register program per query
        for (int q : general_q) {
            int K = 0;
            for (int t = 0; t < qd[q].d; ++t) K = std::max(K, hr[qd[q].rep_base + t].kprimes);
            if (K <= kdone) continue;
            const Handle &h = *hs[q];
            const int d = (int)h.d;
            const uint32_t m = h.m;
            // transform length: m itself, or (m not a power of two) the power of two
            // LM >= 2m - 1 of a zero-padded linear convolution
            const int L = h.pow2 ? h.log2m : ceil_log2(2 * m - 1);
            const uint32_t Mlen = 1u << L;
            const int S = split_of(L);
            const uint32_t *roots = roots_mod(device, L, 0, false, s, &st);
            if (!roots) return st;
            const size_t reg_elems = (size_t)K * d * m;
            uint32_t *M = reinterpret_cast<uint32_t *>(mod_cur);
            mod_cur += align_up((size_t)h.g.n_regs * reg_elems * sizeof(uint32_t));
            uint32_t *padA = nullptr, *padB = nullptr;
            if (!h.pow2) {
                padA = reinterpret_cast<uint32_t *>(mod_cur);
                mod_cur += align_up((size_t)K * d * Mlen * sizeof(uint32_t));
                padB = reinterpret_cast<uint32_t *>(mod_cur);
                mod_cur += align_up((size_t)K * d * Mlen * sizeof(uint32_t));
            }
            const int gx = (int)std::min<size_t>(64, ((size_t)m + 255) / 256);
            const int gxM = (int)std::min<size_t>(256, ((size_t)Mlen + 255) / 256);
            for (const Op &op : h.g.ops) {
                uint32_t *dst = M + (size_t)op.dst * reg_elems;
                switch (op.code) {
                    case OP_LOAD:
                        hipLaunchKernelGGL(k_mod_load, dim3(gx, K * d), dim3(256), 0, s, dst,
                                           rel_counters(h, op.src), m, d, primes);
                        break;
                    case OP_ONES:
                        hipLaunchKernelGGL(k_mod_ones, dim3(gx, K * d), dim3(256), 0, s, dst, m, d, primes);
                        break;
                    case OP_HAD:
                        hipLaunchKernelGGL(k_mod_mul, dim3(gx, K * d), dim3(256), 0, s, dst,
                                           M + (size_t)op.src * reg_elems, m, 0, S, d, primes, 0);
                        break;
                    case OP_CORR: {
                        uint32_t *src = M + (size_t)op.src * reg_elems;
                        if (h.pow2) {
                            st = ntt_forward(nullptr, d, K, src, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                            st = ntt_forward(nullptr, d, K, dst, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                            hipLaunchKernelGGL(k_mod_mul, dim3(gx, K * d), dim3(256), 0, s, dst, src, m, L, S, d,
                                               primes, 1);
                            CSK_HIP(hipGetLastError());
                            st = ntt_inverse(d, K, dst, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                        } else {
                            // src star dst = reverse(src) circularly convolved with dst
                            hipLaunchKernelGGL(k_mod_pad, dim3(gxM, K * d), dim3(256), 0, s, padA, src, m, Mlen, 1);
                            hipLaunchKernelGGL(k_mod_pad, dim3(gxM, K * d), dim3(256), 0, s, padB, dst, m, Mlen, 0);
                            CSK_HIP(hipGetLastError());
                            st = ntt_forward(nullptr, d, K, padA, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                            st = ntt_forward(nullptr, d, K, padB, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                            hipLaunchKernelGGL(k_mod_mul, dim3(gxM, K * d), dim3(256), 0, s, padB, padA, Mlen, L, S, d,
                                               primes, 0);
                            CSK_HIP(hipGetLastError());
                            st = ntt_inverse(d, K, padB, L, S, primes, roots, L, s);
                            if (st != CS_OK) return st;
                            hipLaunchKernelGGL(k_mod_fold, dim3(gx, K * d), dim3(256), 0, s, dst, padB, m, Mlen, d,
                                               primes);
                        }
                        break;
                    }
                    default:
                        return fail(CS_EINVAL, "bad op");
                }
                CSK_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_mod_sum, dim3(qd[q].nb, K * d), dim3(kThreads), 0, s,
                               M + (size_t)h.g.result_reg * reg_elems, m, d, primes, qd[q].nb, d_rep, qd[q].rep_base,
                               mod_plane, d_modp);
            CSK_HIP(hipGetLastError());
        }
        fa.stage = 2;
        fa.kcap = kMaxPrimes;
        if (nq <= 256) hipLaunchKernelGGL((k_finalize<2, kFinThreadsFew>), dim3(nq), dim3(kFinThreadsFew), 0, s, fa);
        else hipLaunchKernelGGL((k_finalize<2, kFinThreadsMany>), dim3(nq), dim3(kFinThreadsMany), 0, s, fa);
        CSK_HIP(hipGetLastError());
        CSK_HIP(hipMemcpyAsync(ho, d_outs, nq * sizeof(OutDev), hipMemcpyDeviceToHost, s));
        if (reps_out) CSK_HIP(hipMemcpyAsync(hr, d_rs, n_rep * sizeof(RepDev), hipMemcpyDeviceToHost, s));
        CSK_HIP(hipStreamSynchronize(s));
    }
    for (int q = 0; q < nq; ++q) {
        cs_estimate_t &o = outs[q];
        o.value = ho[q].value;
        o.exact = ho[q].exact;
        o.fits_i64 = ho[q].fits;
        o.value_i64 = ho[q].fits ? ho[q].lo : 0;
        o.d = qd[q].d;
        o.n_modular = ho[q].n_modular;
        if (reps_out) {
            const cs_reps_t &R = reps_out[q];
            for (int t = 0; t < qd[q].d; ++t) {
                const RepDev &x = hr[qd[q].rep_base + t];
                if (R.value) R.value[t] = x.value;
                if (R.lo) R.lo[t] = x.lo;
                if (R.hi) R.hi[t] = x.hi;
                if (R.exact) R.exact[t] = x.exact;
                if (R.bound) R.bound[t] = x.bound;
            }
        }
    }
    return CS_OK;
}

void release_work(EstimateWork &w)
{
    if (w.buf) hipFree(w.buf);
    if (w.mod) hipFree(w.mod);
    if (w.host) hipHostFree(w.host);
    if (w.ev_upload) hipEventDestroy(w.ev_upload);
    if (w.side) hipStreamDestroy(w.side);
    if (w.ev_fork) hipEventDestroy(w.ev_fork);
    if (w.ev_join) hipEventDestroy(w.ev_join);
    w = EstimateWork{};
}

cs_status estimate_run(Handle &h, hipStream_t s, cs_estimate_t *out, const cs_reps_t *reps)
{
    Handle *hp = &h;
    return estimate_batch(&hp, 1, s, out, reps, h.work, nullptr);
}

cs_status estimate_run_async(Handle &h, hipStream_t s, cs_estimate_t *out)
{
    Handle *hp = &h;
    return estimate_batch(&hp, 1, s, nullptr, nullptr, h.work, out);
}

}  // namespace csk

namespace csk {
namespace {

// Synthetic int64 vectors for timing transforms: a SplitMix64 mix of the index, shifted
// into a sketch-like magnitude.
__global__ void k_tune_fill(int64_t *x, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        x[i] = (int64_t)(z ^ (z >> 31)) >> 40;
    }
}

// flag |= spectrum a (row length 2^Sa) differs from b (2^Sb) at some frequency
__global__ void k_tune_cmp(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b, int n_vec, int log2m,
                           int Sa, int Sb, unsigned int *flag)
{
    const size_t m = (size_t)1 << log2m;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n_vec * m;
         i += (size_t)gridDim.x * blockDim.x) {
        const size_t v = i >> log2m;
        const uint32_t f = (uint32_t)(i & (m - 1));
        if (a[v * m + freq_pos(f, log2m, Sa)] != b[v * m + freq_pos(f, log2m, Sb)]) atomicOr(flag, 1u);
    }
}

__global__ void k_tune_flag0(unsigned int *p) { *p = 0u; }

}  // namespace
}  // namespace csk

extern "C" cs_status cs_tune_transform(int32_t log2m, int32_t n_vec, void *stream, cs_tune_report *out)
{
    using namespace csk;
    if (!out) return fail(CS_EINVAL, "null report");
    if (log2m <= 12 || log2m > kMaxLog2N) return fail(CS_EINVAL, "two-pass transform lengths are 2^13..2^21");
    if (n_vec < 1 || n_vec > 4096) return fail(CS_EINVAL, "n_vec must be in [1, 4096]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int device = 0;
    CSK_HIP(hipGetDevice(&device));
    cs_status st = CS_OK;
    const double *tw = twiddles_f64(device, log2m, s, &st);
    if (!tw) return st;
    const uint32_t *roots = roots_mod(device, log2m, 0, false, s, &st);
    if (!roots) return st;
    PrimeDev *primes = nullptr;
    if ((st = device_primes(device, s, &primes)) != CS_OK) return st;
    const size_t m = (size_t)1 << log2m;
    const size_t elems = (size_t)n_vec * m;
    int64_t *src = nullptr;
    double2 *Z = nullptr;
    uint32_t *N = nullptr, *Nref = nullptr;
    void **ptrs = nullptr;
    unsigned int *flag = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (src) (void)hipFree(src);
        if (Z) (void)hipFree(Z);
        if (N) (void)hipFree(N);
        if (Nref) (void)hipFree(Nref);
        if (ptrs) (void)hipFree(ptrs);
        if (flag) (void)hipFree(flag);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    // packed pairs: vector v's real part is vector 2v of src, its imaginary part 2v + 1
    if (hipMalloc(&src, 2 * elems * sizeof(int64_t)) != hipSuccess || hipMalloc(&Z, elems * sizeof(double2)) != hipSuccess ||
        hipMalloc(&N, elems * sizeof(uint32_t)) != hipSuccess || hipMalloc(&Nref, elems * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&ptrs, 3 * (size_t)n_vec * sizeof(void *)) != hipSuccess ||
        hipMalloc(&flag, sizeof(unsigned int)) != hipSuccess) {
        cleanup();
        return fail(CS_ENOMEM, "transform tuning buffers");
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(CS_EDEVICE, "transform tuning events");
    }
    std::vector<const int64_t *> tab(3 * (size_t)n_vec);
    for (int v = 0; v < n_vec; ++v) {
        tab[v] = src + (size_t)(2 * v) * m;               // fp64: real parts
        tab[n_vec + v] = src + (size_t)(2 * v + 1) * m;   // fp64: imaginary parts
        tab[2 * n_vec + v] = src + (size_t)v * m;         // NTT: one sketch per vector
    }
    hipLaunchKernelGGL(k_tune_fill, dim3(4096), dim3(256), 0, s, src, 2 * elems);
    if (hipMemcpyAsync(ptrs, tab.data(), tab.size() * sizeof(void *), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return fail(CS_EDEVICE, "transform tuning inputs");
    }
    const int64_t *const *re = reinterpret_cast<const int64_t *const *>(ptrs);
    const int64_t *const *im = re + n_vec;
    const int64_t *const *nt = re + 2 * n_vec;
    const int S0 = default_split_bits(log2m);
    std::memset(out, 0, sizeof(*out));
    out->best = -1;
    float best_ms = 0.0f;
    // the default split first: its number-theoretic spectrum is the reference
    std::vector<int> cand{S0};
    for (int S = 10; S <= 12; ++S)
        if (S != S0 && split_ok(log2m, S)) cand.push_back(S);
    for (size_t ci = 0; ci < cand.size() && st == CS_OK; ++ci) {
        const int S = cand[ci];
        cs_tune_candidate &o = out->cand[ci];
        o.strategy = CS_TUNE_TRANSFORM_SPLIT;
        o.grid_blocks = S;
        o.flags = 0;
        o.valid = 0;
        o.ms = -1.0f;
        uint32_t *dst = ci == 0 ? Nref : N;
        if ((st = ntt_forward(nt, n_vec, 1, dst, log2m, S, primes, roots, log2m, s)) != CS_OK) break;
        if (ci > 0) {
            unsigned int hflag = 0;
            hipLaunchKernelGGL(k_tune_flag0, dim3(1), dim3(1), 0, s, flag);
            hipLaunchKernelGGL(k_tune_cmp, dim3(4096), dim3(256), 0, s, N, Nref, n_vec, log2m, S, S0, flag);
            if (hipMemcpyAsync(&hflag, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = fail(CS_EDEVICE, "transform tuning: compare");
                break;
            }
            if (hflag) {
                o.valid = -1;
                continue;
            }
        }
        float t[3];
        bool ok = true;
        for (int r = 0; r < 3 && ok; ++r)
            ok = hipEventRecord(e0, s) == hipSuccess &&
                 fft_f64_forward(re, im, n_vec, Z, log2m, S, reinterpret_cast<const double2 *>(tw), log2m, s) == CS_OK &&
                 ntt_forward(nt, n_vec, 1, N, log2m, S, primes, roots, log2m, s) == CS_OK &&
                 hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        if (!ok) {
            st = fail(CS_EDEVICE, "transform tuning: timing");
            break;
        }
        std::sort(t, t + 3);
        o.ms = t[1];
        o.valid = 1;
        if (out->best < 0 || o.ms < best_ms) {
            out->best = (int32_t)ci;
            best_ms = o.ms;
        }
    }
    out->n = (int32_t)cand.size();
    cleanup();
    if (st != CS_OK) return st;
    if (out->best < 0) return fail(CS_EDEVICE, "transform tuning: no split ran");
    tune_store_split(device, log2m, out->cand[out->best].grid_blocks, best_ms);
    return CS_OK;
}
