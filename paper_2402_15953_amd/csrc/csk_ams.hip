// AMS multi-join sketch (Eq. 1, after Dobra et al.), the baseline the convolution sketch
// is compared with: every counter j of repetition t has its own degree-3 sign
// polynomial per join, so each tuple adds Delta times the product of its joins' signs
// to all d x m counters of its relation (O(d m) per tuple), and the estimate of a
// repetition is X_t = (1/m) sum_j prod_k c_{k,t,j} (Thm. 2.3), median over t.
//
// Update: a workgroup owns 256 counters of one repetition and a chunk of the tuples;
// tiles of keys are staged in LDS and read by every lane at the same address, each lane
// evaluates its counter's sign polynomials (Horner over p = 2^61 - 1, exact parity) and
// keeps the sum in a register; one atomic per counter and chunk at the end.
// Estimate: per repetition, sum_j of the r-fold products in wrapping 128-bit integers
// beside an fp64 bound of sum_j prod_k |c|; the 128-bit sum is the exact numerator
// m X_t whenever the bound stays below 2^126.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "csk_handle.h"
#include "csk_hash.h"
#include "csk_internal.h"

namespace csk {

constexpr int kAmsBlock = 256;
constexpr int kAmsTile = 1024;  // tuples staged in LDS at a time
constexpr int kAmsMaxJoins = 8;  // joins of one relation held in registers

struct AmsHandle {
    int device = 0;
    uint32_t m = 0, d = 0;
    uint64_t seed = 0;
    GraphPlan g;
    std::vector<uint64_t> coef;          // [d][m][n_edge][4]
    int64_t *counters = nullptr;         // [r][d][m]
    uint64_t *coef_dev = nullptr;        // per relation [d][m][4 * joins], concatenated
    std::vector<size_t> coef_off;        // offset of relation k's table
    std::vector<int32_t> joins;          // joins of relation k
    std::vector<std::vector<int8_t>> join_col;  // key column of each join
    void *work = nullptr;                // estimate partials
    size_t work_bytes = 0;
    void *host = nullptr;                // pinned staging of the partials
    size_t host_bytes = 0;
};

}  // namespace csk

struct cs_ams {
    csk::AmsHandle h;
};

namespace csk {
namespace {

struct JoinCols {
    int8_t col[kAmsMaxJoins];
};

// One relation: counters j of repetition t = blockIdx.y, tuples of chunk blockIdx.z.
template <int NJ>
__global__ __launch_bounds__(kAmsBlock) void k_ams_update(const uint32_t *__restrict__ keys, int n_cols,
                                                          const int64_t *__restrict__ weights, uint64_t n,
                                                          uint64_t chunk, const uint64_t *__restrict__ coef,
                                                          JoinCols jc, uint32_t m, unsigned long long *sketch)
{
    __shared__ uint32_t s_k[kAmsTile * kMaxCols];
    __shared__ int64_t s_w[kAmsTile];
    const uint32_t j = blockIdx.x * kAmsBlock + threadIdx.x;
    const uint32_t t = blockIdx.y;
    const bool live = j < m;
    uint64_t a[NJ][4];
    {
        const uint64_t *cf = coef + ((size_t)t * m + (live ? j : 0)) * (4 * NJ);
#pragma unroll
        for (int q = 0; q < NJ; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) a[q][i] = cf[4 * q + i];
    }
    const uint64_t begin = (uint64_t)blockIdx.z * chunk;
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    uint64_t acc = 0;  // two's complement sum of +-Delta (wraps like the counters)
    for (uint64_t base = begin; base < end; base += kAmsTile) {
        const int cnt = (int)(end - base < (uint64_t)kAmsTile ? end - base : (uint64_t)kAmsTile);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * n_cols; e += kAmsBlock) s_k[e] = keys[base * n_cols + e];
        if (weights)
            for (int e = threadIdx.x; e < cnt; e += kAmsBlock) s_w[e] = weights[base + e];
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            uint32_t neg = 0;
#pragma unroll
            for (int q = 0; q < NJ; ++q) {
                const uint32_t x = s_k[i * n_cols + jc.col[q]];
                neg ^= (uint32_t)hcanon(hstep(hstep(hstep(a[q][3], x, a[q][2]), x, a[q][1]), x, a[q][0])) & 1u;
            }
            const uint64_t w = weights ? (uint64_t)s_w[i] : 1ull;
            acc += neg ? 0ull - w : w;
        }
    }
    if (live) atomicAdd(&sketch[(size_t)t * m + j], (unsigned long long)acc);
}

template <int NJ>
cs_status launch_ams(const uint32_t *keys, int n_cols, const int64_t *weights, uint64_t n, const uint64_t *coef,
                     const JoinCols &jc, uint32_t m, uint32_t d, int64_t *sketch, hipStream_t s)
{
    const uint32_t gx = (m + kAmsBlock - 1) / kAmsBlock;
    // tuple chunks: enough workgroups for a few rounds over the chip, whole tiles each
    const uint64_t tiles = (n + kAmsTile - 1) / kAmsTile;
    uint64_t C = std::max<uint64_t>(1, 2048 / ((uint64_t)gx * d));
    C = std::min<uint64_t>(C, std::min<uint64_t>(tiles, 65535));
    const uint64_t chunk = ((tiles + C - 1) / C) * kAmsTile;
    C = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_ams_update<NJ>, dim3(gx, d, (unsigned)C), dim3(kAmsBlock), 0, s, keys, n_cols, weights, n,
                       chunk, coef, jc, m, reinterpret_cast<unsigned long long *>(sketch));
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

// Per (repetition, block): wrapping 128-bit sum of prod_k c_{k,t,j}, and fp64 sums of
// the products and of their absolute values.
struct AmsPartial {
    unsigned long long lo, hi;
    double abs_sum;
    double sum;
};
constexpr int kAmsEstBlocks = 16;

__global__ __launch_bounds__(kAmsBlock) void k_ams_estimate(const int64_t *__restrict__ counters, int r, uint32_t m,
                                                            uint32_t d, AmsPartial *partials)
{
    __shared__ unsigned long long s_lo[kAmsBlock], s_hi[kAmsBlock];
    __shared__ double s_abs[kAmsBlock], s_f[kAmsBlock];
    const uint32_t t = blockIdx.y;
    unsigned __int128 sum = 0;
    double abs_sum = 0.0, fsum = 0.0;
    for (uint32_t j = blockIdx.x * kAmsBlock + threadIdx.x; j < m; j += gridDim.x * kAmsBlock) {
        unsigned __int128 prod = 1;
        double fp = 1.0;
        for (int k = 0; k < r; ++k) {
            const int64_t c = counters[((size_t)k * d + t) * m + j];
            prod *= (unsigned __int128)(__int128)c;
            fp *= (double)c;
        }
        sum += prod;
        abs_sum += fabs(fp);
        fsum += fp;
    }
    s_lo[threadIdx.x] = (unsigned long long)sum;
    s_hi[threadIdx.x] = (unsigned long long)(sum >> 64);
    s_abs[threadIdx.x] = abs_sum;
    s_f[threadIdx.x] = fsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned __int128 tot = 0;
        double at = 0.0, ft = 0.0;
        for (int i = 0; i < kAmsBlock; ++i) {
            tot += ((unsigned __int128)s_hi[i] << 64) | s_lo[i];
            at += s_abs[i];
            ft += s_f[i];
        }
        AmsPartial &p = partials[(size_t)t * gridDim.x + blockIdx.x];
        p.lo = (unsigned long long)tot;
        p.hi = (unsigned long long)(tot >> 64);
        p.abs_sum = at;
        p.sum = ft;
    }
}

__global__ void k_ams_zero(int64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

double i128_to_double_host(__int128 x)
{
    const bool neg = x < 0;
    const unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)x : (unsigned __int128)x;
    const double v = (double)(uint64_t)(u >> 64) * 18446744073709551616.0 + (double)(uint64_t)u;
    return neg ? -v : v;
}

}  // namespace
}  // namespace csk

using namespace csk;

extern "C" {

cs_status cs_ams_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, cs_ams **out)
{
    if (!out) return fail(CS_EINVAL, "null output handle");
    *out = nullptr;
    if (m < 1 || m > (1u << kMaxLog2M)) return fail(CS_EINVAL, "m must be in [1, 2^20]");
    if (d < 1 || d > (uint32_t)kMaxD) return fail(CS_EINVAL, "d must be in [1, 64]");
    cs_ams *hs = new (std::nothrow) cs_ams();
    if (!hs) return fail(CS_ENOMEM, "host allocation failed");
    AmsHandle &h = hs->h;
    cs_status st = analyze_graph(graph, &h.g);
    if (st != CS_OK) {
        delete hs;
        return st;
    }
    h.m = m;
    h.d = d;
    h.seed = seed;
    if (hipGetDevice(&h.device) != hipSuccess) {
        delete hs;
        return fail(CS_EDEVICE, "no HIP device");
    }
    const int E = h.g.n_edge, r = h.g.n_rel;
    // Eq. 1's sign polynomials: order t, j, join, a0..a3 of the seeded stream
    h.coef.resize((size_t)d * m * E * 4);
    SplitMix64 rng{seed};
    for (auto &c : h.coef) c = rng.coef();
    // per relation, in key-column order: the joins at each column's attribute
    std::vector<uint64_t> tab;
    h.coef_off.resize(r);
    h.joins.resize(r);
    h.join_col.resize(r);
    for (int k = 0; k < r; ++k) {
        std::vector<int> eid;
        for (size_t c = 0; c < h.g.omega[k].size(); ++c) {
            const int u = h.g.omega[k][c];
            for (int e : h.g.gamma_edge[u]) {
                eid.push_back(e);
                h.join_col[k].push_back((int8_t)c);
            }
        }
        if (eid.empty() || (int)eid.size() > kAmsMaxJoins) {
            delete hs;
            return fail(CS_EINVAL, "AMS baseline: every relation needs 1 to 8 joins");
        }
        h.joins[k] = (int32_t)eid.size();
        h.coef_off[k] = tab.size();
        for (uint32_t t = 0; t < d; ++t)
            for (uint32_t j = 0; j < m; ++j)
                for (int e : eid)
                    for (int i = 0; i < 4; ++i) tab.push_back(h.coef[(((size_t)t * m + j) * E + e) * 4 + i]);
    }
    const size_t cbytes = (size_t)r * d * m * sizeof(int64_t);
    if (hipMalloc(&h.counters, cbytes) != hipSuccess) {
        delete hs;
        return fail(CS_ENOMEM, "AMS counters");
    }
    if (hipMalloc(&h.coef_dev, tab.size() * sizeof(uint64_t)) != hipSuccess) {
        (void)hipFree(h.counters);
        delete hs;
        return fail(CS_ENOMEM, "AMS coefficients");
    }
    if (hipMemcpy(h.coef_dev, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h.counters, 0, cbytes) != hipSuccess) {
        (void)hipFree(h.counters);
        (void)hipFree(h.coef_dev);
        delete hs;
        return fail(CS_EDEVICE, "AMS initialisation");
    }
    *out = hs;
    return CS_OK;
}

cs_status cs_ams_destroy(cs_ams *hs)
{
    if (!hs) return CS_OK;
    AmsHandle &h = hs->h;
    (void)hipDeviceSynchronize();
    if (h.counters) (void)hipFree(h.counters);
    if (h.coef_dev) (void)hipFree(h.coef_dev);
    if (h.work) (void)hipFree(h.work);
    if (h.host) (void)hipHostFree(h.host);
    delete hs;
    return CS_OK;
}

cs_status cs_ams_update(cs_ams *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                        void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    AmsHandle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n == 0) return CS_OK;
    if (!keys) return fail(CS_EINVAL, "null keys");
    {
        cs_status chk = check_device_array(keys, n * h.g.omega[rel].size() * sizeof(uint32_t), h.device, "keys");
        if (chk == CS_OK && weights) chk = check_device_array(weights, n * sizeof(int64_t), h.device, "weights");
        if (chk != CS_OK) return chk;
    }
    const int n_cols = (int)h.g.omega[rel].size();
    JoinCols jc{};
    for (int q = 0; q < h.joins[rel]; ++q) jc.col[q] = h.join_col[rel][q];
    const uint64_t *cf = h.coef_dev + h.coef_off[rel];
    int64_t *sk = h.counters + (size_t)rel * h.d * h.m;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (h.joins[rel]) {
        case 1: return launch_ams<1>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 2: return launch_ams<2>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 3: return launch_ams<3>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 4: return launch_ams<4>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 5: return launch_ams<5>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 6: return launch_ams<6>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 7: return launch_ams<7>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        case 8: return launch_ams<8>(keys, n_cols, weights, n, cf, jc, h.m, h.d, sk, s);
        default: return fail(CS_EINVAL, "unsupported join count");
    }
}

cs_status cs_ams_reset(cs_ams *hs, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    AmsHandle &h = hs->h;
    const size_t n = (size_t)h.g.n_rel * h.d * h.m;
    hipLaunchKernelGGL(k_ams_zero, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h.counters, n);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

cs_status cs_ams_estimate(cs_ams *hs, void *stream, cs_ams_estimate_t *out, int64_t *rep_lo, int64_t *rep_hi,
                          int32_t *rep_exact)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    AmsHandle &h = hs->h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = (int)std::min<uint32_t>(kAmsEstBlocks, (h.m + kAmsBlock - 1) / kAmsBlock);
    const size_t bytes = (size_t)h.d * nb * sizeof(AmsPartial);
    if (h.work_bytes < bytes) {
        CSK_HIP(hipStreamSynchronize(s));
        if (h.work) (void)hipFree(h.work);
        h.work = nullptr;
        h.work_bytes = 0;
        if (hipMalloc(&h.work, bytes) != hipSuccess) return fail(CS_ENOMEM, "AMS estimate partials");
        h.work_bytes = bytes;
    }
    if (h.host_bytes < bytes) {
        if (h.host) (void)hipHostFree(h.host);
        h.host = nullptr;
        h.host_bytes = 0;
        if (hipHostMalloc(&h.host, bytes, hipHostMallocDefault) != hipSuccess)
            return fail(CS_ENOMEM, "AMS estimate staging");
        h.host_bytes = bytes;
    }
    AmsPartial *dp = static_cast<AmsPartial *>(h.work);
    hipLaunchKernelGGL(k_ams_estimate, dim3(nb, h.d), dim3(kAmsBlock), 0, s, h.counters, h.g.n_rel, h.m, h.d, dp);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipMemcpyAsync(h.host, dp, bytes, hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    const AmsPartial *hp = static_cast<const AmsPartial *>(h.host);
    // per repetition: exact when the bound on |S_t| stays below 2^126.  The fp64 sum of
    // |prod| is below the true sum by at most its roundings: r for the conversions and
    // products of each term, and one per addition on a term's path (its thread's terms,
    // the block's 256 partials, the nb block partials), each relative u = 2^-53.
    const double u = 0x1p-53;
    const double slack = 1.0 + (2.0 * h.g.n_rel + (double)h.m + nb + kAmsBlock) * u * 1.01;
    std::vector<__int128> num(h.d);
    std::vector<int> ex(h.d);
    std::vector<double> val(h.d);
    for (uint32_t t = 0; t < h.d; ++t) {
        unsigned __int128 tot = 0;
        double bound = 0.0, fsum = 0.0;
        for (int b = 0; b < nb; ++b) {
            const AmsPartial &p = hp[(size_t)t * nb + b];
            tot += ((unsigned __int128)p.hi << 64) | p.lo;
            bound += p.abs_sum;
            fsum += p.sum;
        }
        bound *= slack;
        num[t] = (__int128)tot;
        ex[t] = std::isfinite(bound) && bound < 0x1p126;
        val[t] = (ex[t] ? i128_to_double_host(num[t]) : fsum) / (double)h.m;
        if (rep_lo) rep_lo[t] = (int64_t)(uint64_t)tot;
        if (rep_hi) rep_hi[t] = (int64_t)(uint64_t)(tot >> 64);
        if (rep_exact) rep_exact[t] = ex[t];
    }
    // lower median: by rank of the exact numerators when every S_t is exact, else of the
    // fp64 values; the repetition index breaks ties
    int all = 1;
    for (uint32_t t = 0; t < h.d; ++t) all &= ex[t];
    out->exact = all;
    out->num_lo = out->num_hi = 0;
    for (uint32_t t = 0; t < h.d; ++t) {
        uint32_t rank = 0;
        for (uint32_t i = 0; i < h.d; ++i) {
            const bool less = all ? num[i] < num[t] : val[i] < val[t];
            const bool same = all ? num[i] == num[t] : val[i] == val[t];
            rank += less || (same && i < t);
        }
        if (rank == (h.d - 1) / 2) {
            out->median_rep = (int32_t)t;
            out->value = val[t];
            if (all) {
                out->num_lo = (int64_t)(uint64_t)(unsigned __int128)num[t];
                out->num_hi = (int64_t)(uint64_t)((unsigned __int128)num[t] >> 64);
            }
        }
    }
    return CS_OK;
}

cs_status cs_ams_read(const cs_ams *hs, int32_t rel, int64_t *host_out)
{
    if (!hs || !host_out) return fail(CS_EINVAL, "null argument");
    const AmsHandle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    CSK_HIP(hipDeviceSynchronize());
    CSK_HIP(hipMemcpy(host_out, h.counters + (size_t)rel * h.d * h.m, (size_t)h.d * h.m * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    return CS_OK;
}

cs_status cs_ams_coefficients(const cs_ams *hs, uint64_t *host_out)
{
    if (!hs || !host_out) return fail(CS_EINVAL, "null argument");
    std::memcpy(host_out, hs->h.coef.data(), hs->h.coef.size() * sizeof(uint64_t));
    return CS_OK;
}

}  // extern "C"
