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

// ---------------------------------------------------------------- kernels

// Sum of squares and sum of absolute values of each sketch vector (fp64), per block.
__global__ __launch_bounds__(kThreads) void k_norms(const int64_t *__restrict__ sk, int log2m, int nb,
                                                    double *partials)
{
    __shared__ double sh[kThreads / 64];
    const int64_t m = (int64_t)1 << log2m;
    const int64_t *c = sk + (size_t)blockIdx.y * m;
    double s2 = 0.0, s1 = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < m; j += (int64_t)nb * kThreads) {
        const double v = (double)c[j];
        s2 += v * v;
        s1 += fabs(v);
    }
    const double a = block_sum(s2, sh);
    const double b = block_sum(s1, sh);
    if (threadIdx.x == 0) {
        double *o = partials + ((size_t)blockIdx.y * nb + blockIdx.x) * 2;
        o[0] = a;
        o[1] = b;
    }
}

// 128-bit inner product of c_0[t] and c_1[t], per block.
__global__ __launch_bounds__(kThreads) void k_dot(const int64_t *__restrict__ c0, const int64_t *__restrict__ c1,
                                                  int log2m, int nb, unsigned long long *partials)
{
    __shared__ unsigned __int128 sh[kThreads];
    const int64_t m = (int64_t)1 << log2m;
    const int t = blockIdx.y;
    const int64_t *a = c0 + (size_t)t * m;
    const int64_t *b = c1 + (size_t)t * m;
    __int128 acc = 0;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < m; j += (int64_t)nb * kThreads)
        acc += (__int128)a[j] * (__int128)b[j];
    sh[threadIdx.x] = (unsigned __int128)acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long *o = partials + ((size_t)t * nb + blockIdx.x) * 2;
        o[0] = (unsigned long long)(uint64_t)sh[0];
        o[1] = (unsigned long long)(uint64_t)(sh[0] >> 64);
    }
}

// fp64 spectral product-reduce.  vec_of / part_of [d][r]: packed vector and half
// (0: real input, 1: imaginary input) holding relation k's repetition t.
// partials [d][nb][2 + r]: sum Re(term), sum |Re|+|Im| of terms, max |C_k| per relation.
__global__ __launch_bounds__(kThreads) void k_spec_f64(const double2 *__restrict__ Z, int log2m, int r,
                                                       const int32_t *__restrict__ vec_of,
                                                       const int32_t *__restrict__ part_of, uint32_t conj_mask,
                                                       int nb, double *partials)
{
    __shared__ double sh[kThreads / 64];
    const uint32_t m = 1u << log2m;
    const int t = blockIdx.y;
    double acc = 0.0, acc_abs = 0.0;
    double mx[kMaxRel];
#pragma unroll
    for (int k = 0; k < kMaxRel; ++k) mx[k] = 0.0;
    for (uint32_t pos = blockIdx.x * kThreads + threadIdx.x; pos < m; pos += (uint32_t)nb * kThreads) {
        const uint32_t f = pos_freq(pos, log2m);
        const uint32_t npos = freq_pos((m - f) & (m - 1), log2m);
        double pr = 1.0, pi = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxRel; ++k) {
            if (k < r) {
                const double2 *zv = Z + (size_t)vec_of[t * r + k] * m;
                const double2 a = zv[pos], b = zv[npos];
                double cr, ci;
                if (part_of[t * r + k] == 0) {
                    cr = 0.5 * (a.x + b.x);
                    ci = 0.5 * (a.y - b.y);
                } else {
                    cr = 0.5 * (a.y + b.y);
                    ci = 0.5 * (b.x - a.x);
                }
                if ((conj_mask >> k) & 1u) ci = -ci;
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
    double *o = partials + ((size_t)t * nb + blockIdx.x) * (2 + r);
    const double s0 = block_sum(acc, sh);
    if (threadIdx.x == 0) o[0] = s0;
    const double s1 = block_sum(acc_abs, sh);
    if (threadIdx.x == 0) o[1] = s1;
    for (int k = 0; k < r; ++k) {
        const double mk = block_max(mx[k], sh);
        if (threadIdx.x == 0) o[2 + k] = mk;
    }
}

// Modular spectral product-reduce over buffers [K][r*d][m] (vector (i, k, t) at
// i * r * d + k * d + t).  partials [K][d][nb] (uint32 residues, Montgomery form).
__global__ __launch_bounds__(kThreads) void k_spec_mod(const uint32_t *__restrict__ N, int log2m, int r, int d,
                                                       uint32_t conj_mask, const PrimeDev *__restrict__ primes,
                                                       int nb, uint32_t *partials)
{
    __shared__ uint32_t sh[kThreads];
    const uint32_t m = 1u << log2m;
    const int t = blockIdx.y, pi = blockIdx.z;
    const PrimeDev P = primes[pi];
    const RingM R{P.p, P.pinv_neg};
    const uint32_t *base = N + (size_t)pi * r * d * m;
    uint32_t acc = 0;
    for (uint32_t pos = blockIdx.x * kThreads + threadIdx.x; pos < m; pos += (uint32_t)nb * kThreads) {
        const uint32_t f = pos_freq(pos, log2m);
        const uint32_t npos = freq_pos((m - f) & (m - 1), log2m);
        uint32_t prod = P.one;
        for (int k = 0; k < r; ++k) {
            const uint32_t *v = base + ((size_t)k * d + t) * m;
            prod = R.mul(prod, ((conj_mask >> k) & 1u) ? v[npos] : v[pos]);
        }
        acc = R.add(acc, prod);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = R.add(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[((size_t)pi * d + t) * nb + blockIdx.x] = sh[0];
}

// ---- general plan register operations, buffers [K][d][m] per register

__global__ void k_mod_load(uint32_t *reg, const int64_t *__restrict__ sk, int log2m, int d,
                           const PrimeDev *__restrict__ primes)
{
    const int64_t m = (int64_t)1 << log2m;
    const int v = blockIdx.y;  // i * d + t
    const PrimeDev P = primes[v / d];
    const RingM R{P.p, P.pinv_neg};
    const int64_t *c = sk + (size_t)(v % d) * m;
    uint32_t *o = reg + (size_t)v * m;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        o[j] = mont_from_i64(R, c[j], P.r2, P.r3, P.neg2_64);
}

__global__ void k_mod_ones(uint32_t *reg, int log2m, int d, const PrimeDev *__restrict__ primes)
{
    const int64_t m = (int64_t)1 << log2m;
    const int v = blockIdx.y;
    const uint32_t one = primes[v / d].one;
    uint32_t *o = reg + (size_t)v * m;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        o[j] = one;
}

// dst = dst o src (time domain) or dst[pos] = src[-f] * dst[f] (frequency domain, the
// pointwise step of the cross-correlation src star dst).
__global__ void k_mod_mul(uint32_t *dst, const uint32_t *__restrict__ src, int log2m, int d,
                          const PrimeDev *__restrict__ primes, int negate_src)
{
    const uint32_t m = 1u << log2m;
    const int v = blockIdx.y;
    const PrimeDev P = primes[v / d];
    const RingM R{P.p, P.pinv_neg};
    uint32_t *o = dst + (size_t)v * m;
    const uint32_t *a = src + (size_t)v * m;
    for (uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x; pos < m; pos += gridDim.x * blockDim.x) {
        uint32_t sp = pos;
        if (negate_src) sp = freq_pos((m - pos_freq(pos, log2m)) & (m - 1), log2m);
        o[pos] = R.mul(o[pos], a[sp]);
    }
}

__global__ __launch_bounds__(kThreads) void k_mod_sum(const uint32_t *__restrict__ reg, int log2m, int d,
                                                      const PrimeDev *__restrict__ primes, int nb,
                                                      uint32_t *partials)
{
    __shared__ uint32_t sh[kThreads];
    const uint32_t m = 1u << log2m;
    const int v = blockIdx.y;  // i * d + t
    const PrimeDev P = primes[v / d];
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
    // partials [K][d][nb]
    if (threadIdx.x == 0) partials[(size_t)v * nb + blockIdx.x] = sh[0];
}

// ---- finalize

struct FinalizeArgs {
    int32_t plan;
    int32_t stage;        // 1: after the fp64 / dot / norms pass; 2: after the modular pass
    int32_t r, d, log2m;
    int32_t nb_norm, nb_spec, nb_mod, nb_dot;
    int32_t n_primes;     // primes used by the modular pass (stage 2)
    int32_t mod_scale_m;  // modular partial sums carry the 1/m factor of the spectral sum
    const double *norms;  // [r*d][nb_norm][2]
    const double *spec;   // [d][nb_spec][2+r]
    const unsigned long long *dot;  // [d][nb_dot][2]
    const uint32_t *modp; // [K][d][nb_mod]
    const int32_t *partner;  // [r*d] sketch index packed with sketch s, -1 none
    const PrimeDev *primes;
    CrtTables crt;
    RepDev *reps;
    OutDev *out;
    double n_eff_spec;    // sequential additions in the spectral sum (rounding bound)
    double n_eff_norm;
};

__global__ void k_finalize(FinalizeArgs a)
{
    const int t = threadIdx.x;
    const double u = 0x1p-53;
    const double m = (double)(1u << a.log2m);
    if (t < a.d) {
        RepDev &rp = a.reps[t];
        if (a.stage == 1) {
            rp.kprimes = 0;
            rp.status = 0;
            rp.window = 0;
            rp.bound = 0.0;
            if (a.plan == CS_PLAN_DOT) {
                unsigned __int128 s = 0;
                for (int b = 0; b < a.nb_dot; ++b) {
                    const unsigned long long *p = a.dot + ((size_t)t * a.nb_dot + b) * 2;
                    s += ((unsigned __int128)p[1] << 64) | p[0];
                }
                const __int128 x = (__int128)s;
                rp.lo = (int64_t)(uint64_t)s;
                rp.hi = (int64_t)(uint64_t)(s >> 64);
                rp.exact = 1;
                rp.value = i128_to_double(x);
                rp.xf = rp.value;
            } else {
                // norms of each relation's sketch at this repetition (upper bounds)
                double s2[kMaxRel], s1[kMaxRel];
                const double up = 1.0 + (a.n_eff_norm + 4.0) * u * 1.01;
                for (int k = 0; k < a.r; ++k) {
                    const int s = k * a.d + t;
                    double q = 0.0, l = 0.0;
                    for (int b = 0; b < a.nb_norm; ++b) {
                        q += a.norms[((size_t)s * a.nb_norm + b) * 2];
                        l += a.norms[((size_t)s * a.nb_norm + b) * 2 + 1];
                    }
                    s2[k] = q * up;
                    s1[k] = l * up;
                }
                if (a.plan == CS_PLAN_SPECTRAL) {
                    double sum = 0.0, sabs = 0.0, mx[kMaxRel];
                    for (int k = 0; k < a.r; ++k) mx[k] = 0.0;
                    for (int b = 0; b < a.nb_spec; ++b) {
                        const double *p = a.spec + ((size_t)t * a.nb_spec + b) * (2 + a.r);
                        sum += p[0];
                        sabs += p[1];
                        for (int k = 0; k < a.r; ++k) mx[k] = fmax(mx[k], p[2 + k]);
                    }
                    const double xf = sum / m;
                    // fp64 FFT error (radix-2 Cooley-Tukey, twiddles within 2u):
                    // ||fl(FFT z) - FFT z||_2 <= kappa sqrt(m) ||z||_2.
                    const double g4 = 4.0 * u / (1.0 - 4.0 * u);
                    const double eta = 2.0 * u + g4 * (1.41421356237309515 + 2.0 * u);
                    const double kappa = 2.0 * (a.log2m + 3) * eta;
                    const double sm = sqrt(m) * (1.0 + 4.0 * u);
                    double e[kMaxRel], N[kMaxRel], M[kMaxRel];
                    for (int k = 0; k < a.r; ++k) {
                        const int s = k * a.d + t;
                        const int ps = a.partner[s];
                        double z2 = s2[k];
                        if (ps >= 0) {
                            // partner's squared norm, recomputed from the norm partials
                            double q = 0.0;
                            for (int b = 0; b < a.nb_norm; ++b) q += a.norms[((size_t)ps * a.nb_norm + b) * 2];
                            z2 += q * up;
                        }
                        e[k] = kappa * sm * sqrt(z2) * (1.0 + 4.0 * u);
                        N[k] = sm * sqrt(s2[k]) * (1.0 + 4.0 * u) + e[k];
                        M[k] = mx[k] * (1.0 + 4.0 * u) + e[k];
                    }
                    double dT = 0.0;
                    for (int k = 0; k < a.r; ++k) {
                        double best = INFINITY;
                        for (int j = 0; j < a.r; ++j) {
                            if (j == k) continue;
                            double v = N[j];
                            for (int i = 0; i < a.r; ++i)
                                if (i != j && i != k) v *= M[i];
                            best = fmin(best, v);
                        }
                        dT += e[k] * best;
                    }
                    const double rho = ((a.r - 1) * 3.0 + a.n_eff_spec + 4.0) * u * 1.01;
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
                            // window around xf when xf fits in int128, else full centered range
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
                    for (int k = 0; k < a.r; ++k) {
                        if (s1[k] == 0.0) zero = true;
                        lb += log2(s1[k]);
                    }
                    rp.exact = 0;
                    rp.value = 0.0;
                    rp.xf = 0.0;
                    if (zero) {
                        rp.exact = 1;
                        rp.lo = rp.hi = 0;
                        rp.value = 0.0;
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
        } else if (rp.kprimes > 0) {  // stage 2: residues -> exact value
            const int K = rp.kprimes;
            uint32_t res[kMaxPrimes], dig[kMaxPrimes];
            for (int i = 0; i < K; ++i) {
                const PrimeDev &P = a.primes[i];
                const RingM R{P.p, P.pinv_neg};
                uint32_t s = 0;
                for (int b = 0; b < a.nb_mod; ++b) s = R.add(s, a.modp[((size_t)i * a.d + t) * a.nb_mod + b]);
                if (a.mod_scale_m) s = R.mul(s, P.minv[a.log2m]);
                res[i] = R.mul(s, 1u);  // out of Montgomery form
            }
            if (a.plan == CS_PLAN_SPECTRAL && rp.window) {
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
    }
    __syncthreads();
    if (t == 0) {
        // median: order by fp64 value, ties between exact values by the integers
        int idx[kMaxD];
        int n_mod = 0;
        for (int i = 0; i < a.d; ++i) {
            idx[i] = i;
            if (a.reps[i].kprimes > 0) ++n_mod;
        }
        for (int i = 1; i < a.d; ++i) {
            const int cur = idx[i];
            int j = i - 1;
            while (j >= 0) {
                const RepDev &A = a.reps[idx[j]];
                const RepDev &B = a.reps[cur];
                bool greater;
                if (A.value != B.value) {
                    greater = A.value > B.value;
                } else if (A.exact && B.exact) {
                    const __int128 xa = (__int128)(((unsigned __int128)(uint64_t)A.hi << 64) | (uint64_t)A.lo);
                    const __int128 xb = (__int128)(((unsigned __int128)(uint64_t)B.hi << 64) | (uint64_t)B.lo);
                    greater = xa > xb;
                } else {
                    greater = false;
                }
                if (!greater) break;
                idx[j + 1] = idx[j];
                --j;
            }
            idx[j + 1] = cur;
        }
        const int med = idx[(a.d - 1) / 2];
        const RepDev &R = a.reps[med];
        a.out->value = R.value;
        a.out->lo = R.lo;
        a.out->hi = R.hi;
        a.out->exact = R.exact;
        const __int128 x = (__int128)(((unsigned __int128)(uint64_t)R.hi << 64) | (uint64_t)R.lo);
        a.out->fits = R.exact && x >= (__int128)INT64_MIN && x <= (__int128)INT64_MAX;
        a.out->n_modular = n_mod;
        a.out->median_rep = med;
    }
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
    const uint64_t step = 1ull << kMaxLog2M;
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
        // generator: p - 1 = c * 2^20
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
            for (int L = 0; L <= kMaxLog2M; ++L) {
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

// ---------------------------------------------------------------- work buffers

struct Work {
    double *norms = nullptr;
    double *spec = nullptr;
    unsigned long long *dot = nullptr;
    uint32_t *modp = nullptr;
    double2 *Z = nullptr;
    uint32_t *modbuf = nullptr;
    int32_t *tables = nullptr;   // pack_re, pack_im, vec_of, part_of, partner, sk_index
    RepDev *reps = nullptr;
    OutDev *out = nullptr;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

const std::vector<PrimeInfo> &ntt_primes()
{
    static const std::vector<PrimeInfo> P = build_primes();
    return P;
}

const double *twiddles_f64(int device, int log2m, hipStream_t s, cs_status *st)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    DeviceTables &T = g_tabs[device];
    auto it = T.tw.find(log2m);
    if (it != T.tw.end()) {
        *st = CS_OK;
        return reinterpret_cast<const double *>(it->second);
    }
    const size_t m = (size_t)1 << log2m;
    std::vector<double2> h(m);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (size_t k = 0; k < m; ++k) {
        const long double ang = -two_pi * (long double)k / (long double)m;
        h[k] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    double2 *dp = nullptr;
    if (hipMalloc(&dp, m * sizeof(double2)) != hipSuccess) {
        *st = fail(CS_ENOMEM, "twiddle table allocation failed");
        return nullptr;
    }
    if (hipMemcpy(dp, h.data(), m * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        *st = fail(CS_EDEVICE, "twiddle upload failed");
        return nullptr;
    }
    (void)s;
    T.tw[log2m] = dp;
    *st = CS_OK;
    return reinterpret_cast<const double *>(dp);
}

const uint32_t *roots_mod(int device, int log2m, int /*prime*/, bool /*inverse*/, hipStream_t s, cs_status *st)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    DeviceTables &T = g_tabs[device];
    auto it = T.roots.find(log2m);
    if (it != T.roots.end()) {
        *st = CS_OK;
        return it->second;
    }
    const auto &P = ntt_primes();
    const size_t m = (size_t)1 << log2m;
    std::vector<uint32_t> h((size_t)kMaxPrimes * 2 * m);
    for (int i = 0; i < kMaxPrimes; ++i) {
        const uint64_t p = P[i].p;
        const uint64_t w = powmod(P[i].g, (p - 1) >> log2m, p);
        const uint64_t wi = powmod(w, p - 2, p);
        const uint64_t R = (1ull << 32) % p;
        for (int dir = 0; dir < 2; ++dir) {
            uint64_t acc = 1;
            const uint64_t step = dir ? wi : w;
            uint32_t *dst = h.data() + ((size_t)(2 * i + dir) << log2m);
            for (size_t k = 0; k < m; ++k) {
                dst[k] = (uint32_t)((unsigned __int128)acc * R % p);
                acc = (unsigned __int128)acc * step % p;
            }
        }
    }
    uint32_t *dp = nullptr;
    if (hipMalloc(&dp, h.size() * sizeof(uint32_t)) != hipSuccess) {
        *st = fail(CS_ENOMEM, "root table allocation failed");
        return nullptr;
    }
    if (hipMemcpy(dp, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        *st = fail(CS_EDEVICE, "root table upload failed");
        return nullptr;
    }
    (void)s;
    T.roots[log2m] = dp;
    *st = CS_OK;
    return dp;
}

cs_status estimate_run(Handle &h, hipStream_t s, cs_estimate_t *out, const cs_reps_t *reps)
{
    const GraphPlan &g = h.g;
    const int r = g.n_rel, d = (int)h.d, L = h.log2m;
    const size_t m = h.m;
    const int plan = g.plan;
    PrimeDev *primes = nullptr;
    cs_status st = device_primes(h.device, s, &primes);
    if (st != CS_OK) return st;

    // block counts: each thread of a reduction handles >= 8 elements
    auto nblocks = [&](size_t len) {
        size_t nb = len / (kThreads * 8);
        if (nb < 1) nb = 1;
        if (nb > 64) nb = 64;
        return (int)nb;
    };
    const int nb = nblocks(m);
    const int n_sk = r * d;
    const int n_vec = (n_sk + 1) / 2;
    int n_regs = g.n_regs > 0 ? g.n_regs : 1;

    // ---- sizes of the work buffers (kMaxPrimes primes reserved for modular buffers)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t o_norms = take((size_t)n_sk * nb * 2 * sizeof(double));
    const size_t o_spec = take((size_t)d * nb * (2 + r) * sizeof(double));
    const size_t o_dot = take((size_t)d * nb * 2 * sizeof(unsigned long long));
    const size_t o_modp = take((size_t)kMaxPrimes * d * nb * sizeof(uint32_t));
    const size_t o_Z = take(plan == CS_PLAN_SPECTRAL ? (size_t)n_vec * m * sizeof(double2) : 0);
    size_t mod_elems = 0;
    const size_t o_tables = take((size_t)(2 * n_vec + 3 * n_sk + n_sk) * sizeof(int32_t));
    const size_t o_reps = take((size_t)d * sizeof(RepDev));
    const size_t o_out = take(sizeof(OutDev));
    const size_t base_bytes = off;
    (void)mod_elems;
    (void)n_regs;
    if (h.work.bytes < base_bytes) {
        if (h.work.buf) hipFree(h.work.buf);
        h.work.buf = nullptr;
        h.work.bytes = 0;
        if (hipMalloc(&h.work.buf, base_bytes) != hipSuccess) return fail(CS_ENOMEM, "estimate workspace");
        h.work.bytes = base_bytes;
    }
    char *wb = static_cast<char *>(h.work.buf);
    Work w;
    w.norms = reinterpret_cast<double *>(wb + o_norms);
    w.spec = reinterpret_cast<double *>(wb + o_spec);
    w.dot = reinterpret_cast<unsigned long long *>(wb + o_dot);
    w.modp = reinterpret_cast<uint32_t *>(wb + o_modp);
    w.Z = reinterpret_cast<double2 *>(wb + o_Z);
    w.tables = reinterpret_cast<int32_t *>(wb + o_tables);
    w.reps = reinterpret_cast<RepDev *>(wb + o_reps);
    w.out = reinterpret_cast<OutDev *>(wb + o_out);

    // ---- host tables: packing of (relation, repetition) sketches into complex vectors
    std::vector<int32_t> tab(2 * n_vec + 3 * n_sk + n_sk, -1);
    int32_t *pack_re = tab.data(), *pack_im = pack_re + n_vec, *vec_of = pack_im + n_vec;
    int32_t *part_of = vec_of + n_sk, *partner = part_of + n_sk, *sk_index = partner + n_sk;
    for (int v = 0; v < n_vec; ++v) {
        pack_re[v] = 2 * v;
        pack_im[v] = 2 * v + 1 < n_sk ? 2 * v + 1 : -1;
    }
    for (int k = 0; k < r; ++k)
        for (int t = 0; t < d; ++t) {
            const int sidx = k * d + t;
            vec_of[t * r + k] = sidx / 2;
            part_of[t * r + k] = sidx % 2;
            const int other = sidx ^ 1;
            partner[sidx] = other < n_sk ? other : -1;
            sk_index[sidx] = sidx;
        }
    int32_t *dtab = w.tables;
    CSK_HIP(hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int32_t *d_pack_re = dtab, *d_pack_im = dtab + n_vec, *d_vec_of = d_pack_im + n_vec;
    const int32_t *d_part_of = d_vec_of + n_sk, *d_partner = d_part_of + n_sk, *d_sk_index = d_partner + n_sk;

    FinalizeArgs fa{};
    fa.plan = plan;
    fa.r = r;
    fa.d = d;
    fa.log2m = L;
    fa.nb_norm = nb;
    fa.nb_spec = nb;
    fa.nb_mod = nb;
    fa.nb_dot = nb;
    fa.norms = w.norms;
    fa.spec = w.spec;
    fa.dot = w.dot;
    fa.modp = w.modp;
    fa.partner = d_partner;
    fa.primes = primes;
    fa.crt = g_crt;
    fa.reps = w.reps;
    fa.out = w.out;
    const double per_thread = std::ceil((double)m / ((double)nb * kThreads));
    fa.n_eff_spec = per_thread + 8.0 + nb;
    fa.n_eff_norm = per_thread + 8.0 + nb;

    // ---- stage 1
    if (plan == CS_PLAN_DOT) {
        const int64_t *c0 = h.counters;
        const int64_t *c1 = h.counters + (size_t)d * m;
        hipLaunchKernelGGL(k_dot, dim3(nb, d), dim3(kThreads), 0, s, c0, c1, L, nb, w.dot);
        CSK_HIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL(k_norms, dim3(nb, n_sk), dim3(kThreads), 0, s, h.counters, L, nb, w.norms);
        CSK_HIP(hipGetLastError());
        if (plan == CS_PLAN_SPECTRAL) {
            const double *tw = twiddles_f64(h.device, L, s, &st);
            if (!tw) return st;
            st = fft_f64_forward(h.counters, d_pack_re, d_pack_im, n_vec, w.Z, L,
                                 reinterpret_cast<const double2 *>(tw), L, s);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_spec_f64, dim3(nb, d), dim3(kThreads), 0, s, w.Z, L, r, d_vec_of, d_part_of,
                               g.conj_mask, nb, w.spec);
            CSK_HIP(hipGetLastError());
        }
    }
    fa.stage = 1;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kMaxD), 0, s, fa);
    CSK_HIP(hipGetLastError());

    std::vector<RepDev> hr(d);
    CSK_HIP(hipMemcpyAsync(hr.data(), w.reps, d * sizeof(RepDev), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    int K = 0;
    for (int t = 0; t < d; ++t) K = std::max(K, hr[t].kprimes);

    // ---- stage 2: modular residues
    if (K > 0) {
        const uint32_t *roots = roots_mod(h.device, L, 0, false, s, &st);
        if (!roots) return st;
        size_t mod_bytes;
        if (plan == CS_PLAN_SPECTRAL) mod_bytes = (size_t)K * n_sk * m * sizeof(uint32_t);
        else mod_bytes = (size_t)g.n_regs * K * d * m * sizeof(uint32_t);
        void *mb = nullptr;
        if (hipMallocAsync(&mb, mod_bytes, s) != hipSuccess) return fail(CS_ENOMEM, "modular workspace");
        uint32_t *M = static_cast<uint32_t *>(mb);
        if (plan == CS_PLAN_SPECTRAL) {
            st = ntt_forward(h.counters, d_sk_index, n_sk, K, M, L, primes, roots, L, s);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_spec_mod, dim3(nb, d, K), dim3(kThreads), 0, s, M, L, r, d, g.conj_mask, primes,
                               nb, w.modp);
            CSK_HIP(hipGetLastError());
            fa.mod_scale_m = 1;
        } else {
            const size_t reg_elems = (size_t)K * d * m;
            const int gx = (int)std::min<size_t>(64, (m + 255) / 256);
            for (const Op &op : g.ops) {
                uint32_t *dst = M + (size_t)op.dst * reg_elems;
                switch (op.code) {
                    case OP_LOAD:
                        hipLaunchKernelGGL(k_mod_load, dim3(gx, K * d), dim3(256), 0, s, dst,
                                           h.counters + (size_t)op.src * d * m, L, d, primes);
                        break;
                    case OP_ONES:
                        hipLaunchKernelGGL(k_mod_ones, dim3(gx, K * d), dim3(256), 0, s, dst, L, d, primes);
                        break;
                    case OP_HAD:
                        hipLaunchKernelGGL(k_mod_mul, dim3(gx, K * d), dim3(256), 0, s, dst,
                                           M + (size_t)op.src * reg_elems, L, d, primes, 0);
                        break;
                    case OP_CORR: {
                        uint32_t *src = M + (size_t)op.src * reg_elems;
                        st = ntt_forward(nullptr, nullptr, d, K, src, L, primes, roots, L, s);
                        if (st != CS_OK) return st;
                        st = ntt_forward(nullptr, nullptr, d, K, dst, L, primes, roots, L, s);
                        if (st != CS_OK) return st;
                        hipLaunchKernelGGL(k_mod_mul, dim3(gx, K * d), dim3(256), 0, s, dst, src, L, d, primes, 1);
                        CSK_HIP(hipGetLastError());
                        st = ntt_inverse(d, K, dst, L, primes, roots, L, s);
                        if (st != CS_OK) return st;
                        break;
                    }
                    default:
                        return fail(CS_EINVAL, "bad op");
                }
                CSK_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_mod_sum, dim3(nb, K * d), dim3(kThreads), 0, s,
                               M + (size_t)g.result_reg * reg_elems, L, d, primes, nb, w.modp);
            CSK_HIP(hipGetLastError());
            fa.mod_scale_m = 0;
        }
        fa.stage = 2;
        fa.n_primes = K;
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kMaxD), 0, s, fa);
        CSK_HIP(hipGetLastError());
        CSK_HIP(hipFreeAsync(mb, s));
    }

    OutDev ho;
    CSK_HIP(hipMemcpyAsync(&ho, w.out, sizeof(OutDev), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipMemcpyAsync(hr.data(), w.reps, d * sizeof(RepDev), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    out->value = ho.value;
    out->exact = ho.exact;
    out->fits_i64 = ho.fits;
    out->value_i64 = ho.fits ? ho.lo : 0;
    out->d = d;
    out->n_modular = ho.n_modular;
    if (reps) {
        for (int t = 0; t < d; ++t) {
            if (reps->value) reps->value[t] = hr[t].value;
            if (reps->lo) reps->lo[t] = hr[t].lo;
            if (reps->hi) reps->hi[t] = hr[t].hi;
            if (reps->exact) reps->exact[t] = hr[t].exact;
            if (reps->bound) reps->bound[t] = hr[t].bound;
        }
    }
    return CS_OK;
}

}  // namespace csk
