// Per-attribute sketches for query optimizers (Sec. 3.4): the optimizer needs the
// sizes of many sub-queries, and a sketch of an attribute can be reused by every
// sub-query that joins that attribute once.  Each attribute u of a base query gets one
// Count sketch [d][m] built with the hash functions of its graph component (a sign
// polynomial of degree 3 and a bin polynomial of degree 1 per repetition), so any two
// attributes of one component estimate their two-relation join by the inner product of
// their sketches (Eq. 5 with r = 2), median over the repetitions.
//
// One pass over a relation's tuples updates the sketches of all its joined attributes:
// the key columns are split into contiguous columns by one gather launch, and each
// column goes through the ordinary update path (the same kernels and strategies as a
// one-column relation of a query).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "csk_handle.h"
#include "csk_internal.h"

namespace csk {

struct AttrHandle {
    int device = 0;
    uint32_t m = 0, d = 0;
    uint64_t seed = 0;
    GraphPlan g;
    std::vector<uint64_t> sign;        // [d][Q][4]
    std::vector<uint64_t> bin;         // [d][Q][2]
    int64_t *counters = nullptr;       // [w][d][m]
    uint64_t *coef_dev = nullptr;      // per component: [d][6] = b0, b1, a0..a3
    uint32_t *columns = nullptr;       // gathered key columns [a][n]
    size_t column_bytes = 0;
    void *work = nullptr;              // estimate partials
    size_t work_bytes = 0;
    void *host = nullptr;              // pinned staging of the partials
    size_t host_bytes = 0;
};

}  // namespace csk

struct cs_attr {
    csk::AttrHandle h;
};

namespace csk {
namespace {

constexpr int kAttrBlock = 256;
constexpr int kAttrDotBlocks = 32;

// [n][a] tuple-major keys -> [a][n] columns
__global__ void k_gather_columns(const uint32_t *__restrict__ keys, int a, uint64_t n, uint32_t *out)
{
    const uint64_t total = n * (uint64_t)a;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = e / a;
        const int c = (int)(e - i * a);
        out[(uint64_t)c * n + i] = keys[e];
    }
}

// Per (repetition, block): wrapping 128-bit sum of x[t][j] * y[t][j], and fp64 sums of
// the products and of their absolute values.
struct DotPartial {
    unsigned long long lo, hi;
    double abs_sum, sum;
};

__global__ __launch_bounds__(kAttrBlock) void k_attr_dot(const int64_t *__restrict__ x, const int64_t *__restrict__ y,
                                                         uint32_t m, DotPartial *partials)
{
    __shared__ unsigned long long s_lo[kAttrBlock], s_hi[kAttrBlock];
    __shared__ double s_a[kAttrBlock], s_f[kAttrBlock];
    const uint32_t t = blockIdx.y;
    const int64_t *xt = x + (size_t)t * m;
    const int64_t *yt = y + (size_t)t * m;
    unsigned __int128 acc = 0;
    double aa = 0.0, ff = 0.0;
    for (uint32_t j = blockIdx.x * kAttrBlock + threadIdx.x; j < m; j += gridDim.x * kAttrBlock) {
        acc += (unsigned __int128)((__int128)xt[j] * (__int128)yt[j]);
        const double p = (double)xt[j] * (double)yt[j];
        aa += fabs(p);
        ff += p;
    }
    s_lo[threadIdx.x] = (unsigned long long)acc;
    s_hi[threadIdx.x] = (unsigned long long)(acc >> 64);
    s_a[threadIdx.x] = aa;
    s_f[threadIdx.x] = ff;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned __int128 tot = 0;
        double at = 0.0, ft = 0.0;
        for (int i = 0; i < kAttrBlock; ++i) {
            tot += ((unsigned __int128)s_hi[i] << 64) | s_lo[i];
            at += s_a[i];
            ft += s_f[i];
        }
        DotPartial &p = partials[(size_t)t * gridDim.x + blockIdx.x];
        p.lo = (unsigned long long)tot;
        p.hi = (unsigned long long)(tot >> 64);
        p.abs_sum = at;
        p.sum = ft;
    }
}

__global__ void k_attr_zero(int64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

double i128_to_double_attr(__int128 x)
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

cs_status cs_attr_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, cs_attr **out)
{
    if (!out) return fail(CS_EINVAL, "null output handle");
    *out = nullptr;
    if (m < 2 || m > (1u << kMaxLog2M)) return fail(CS_EINVAL, "m must be in [2, 2^20]");
    if (d < 1 || d > (uint32_t)kMaxD) return fail(CS_EINVAL, "d must be in [1, 64]");
    cs_attr *hs = new (std::nothrow) cs_attr();
    if (!hs) return fail(CS_ENOMEM, "host allocation failed");
    AttrHandle &h = hs->h;
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
    const int Q = h.g.n_comp, w = h.g.n_attr;
    // per repetition, per component: sign a0..a3, then bin b0, b1
    h.sign.resize((size_t)d * Q * 4);
    h.bin.resize((size_t)d * Q * 2);
    SplitMix64 rng{seed};
    for (uint32_t t = 0; t < d; ++t)
        for (int q = 0; q < Q; ++q) {
            for (int i = 0; i < 4; ++i) h.sign[((size_t)t * Q + q) * 4 + i] = rng.coef();
            for (int i = 0; i < 2; ++i) h.bin[((size_t)t * Q + q) * 2 + i] = rng.coef();
        }
    // update-kernel order for one column with one join: b0, b1, a0..a3 per repetition
    std::vector<uint64_t> tab((size_t)Q * d * 6);
    for (int q = 0; q < Q; ++q)
        for (uint32_t t = 0; t < d; ++t) {
            uint64_t *o = tab.data() + ((size_t)q * d + t) * 6;
            o[0] = h.bin[((size_t)t * Q + q) * 2 + 0];
            o[1] = h.bin[((size_t)t * Q + q) * 2 + 1];
            for (int i = 0; i < 4; ++i) o[2 + i] = h.sign[((size_t)t * Q + q) * 4 + i];
        }
    const size_t cbytes = (size_t)w * d * m * sizeof(int64_t);
    if (hipMalloc(&h.counters, cbytes) != hipSuccess) {
        delete hs;
        return fail(CS_ENOMEM, "attribute counters");
    }
    if (hipMalloc(&h.coef_dev, tab.size() * sizeof(uint64_t)) != hipSuccess) {
        (void)hipFree(h.counters);
        delete hs;
        return fail(CS_ENOMEM, "attribute coefficients");
    }
    if (hipMemcpy(h.coef_dev, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h.counters, 0, cbytes) != hipSuccess) {
        (void)hipFree(h.counters);
        (void)hipFree(h.coef_dev);
        delete hs;
        return fail(CS_EDEVICE, "attribute sketch initialisation");
    }
    *out = hs;
    return CS_OK;
}

cs_status cs_attr_destroy(cs_attr *hs)
{
    if (!hs) return CS_OK;
    AttrHandle &h = hs->h;
    (void)hipDeviceSynchronize();
    if (h.counters) (void)hipFree(h.counters);
    if (h.coef_dev) (void)hipFree(h.coef_dev);
    if (h.columns) (void)hipFree(h.columns);
    if (h.work) (void)hipFree(h.work);
    if (h.host) (void)hipHostFree(h.host);
    delete hs;
    return CS_OK;
}

cs_status cs_attr_update(cs_attr *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                         int32_t flags, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    AttrHandle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n == 0) return CS_OK;
    if (!keys) return fail(CS_EINVAL, "null keys");
    {
        cs_status chk = check_device_array(keys, n * h.g.omega[rel].size() * sizeof(uint32_t), h.device, "keys");
        if (chk == CS_OK && weights) chk = check_device_array(weights, n * sizeof(int64_t), h.device, "weights");
        if (chk != CS_OK) return chk;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::vector<int32_t> &cols = h.g.omega[rel];
    const int a = (int)cols.size();
    const uint32_t *colp = keys;
    if (a > 1) {
        const size_t need = (size_t)a * n * sizeof(uint32_t);
        if (h.column_bytes < need) {
            CSK_HIP(hipStreamSynchronize(s));
            if (h.columns) (void)hipFree(h.columns);
            h.columns = nullptr;
            h.column_bytes = 0;
            if (hipMalloc(&h.columns, need) != hipSuccess) return fail(CS_ENOMEM, "attribute column buffer");
            h.column_bytes = need;
        }
        const uint64_t total = n * (uint64_t)a;
        hipLaunchKernelGGL(k_gather_columns, dim3((unsigned)std::min<uint64_t>((total + 255) / 256, 16384)),
                           dim3(256), 0, s, keys, a, n, h.columns);
        CSK_HIP(hipGetLastError());
        colp = h.columns;
    }
    for (int c = 0; c < a; ++c) {
        const int u = cols[c];
        const int q = h.g.psi[u];
        UpdateArgs ua{};
        ua.keys = colp + (size_t)c * (a > 1 ? n : 0);
        ua.weights = weights;
        ua.n = n;
        ua.coef = h.coef_dev + (size_t)q * h.d * 6;
        ua.sketch = reinterpret_cast<uint64_t *>(h.counters + (size_t)u * h.d * h.m);
        ua.m = h.m;
        ua.d = (int32_t)h.d;
        std::memset(&ua.plan, 0, sizeof(ua.plan));
        ua.plan.n_cols = 1;
        ua.plan.n_edges[0] = 1;
        ua.plan.coef_per_rep = 6;
        ua.unit_weights = (flags & CS_UPDATE_UNIT_WEIGHTS) != 0;
        const cs_status st = launch_update(ua, CS_UPDATE_AUTO, 0, s);
        if (st != CS_OK) return st;
    }
    return CS_OK;
}

cs_status cs_attr_reset(cs_attr *hs, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    AttrHandle &h = hs->h;
    const size_t n = (size_t)h.g.n_attr * h.d * h.m;
    hipLaunchKernelGGL(k_attr_zero, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h.counters, n);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

cs_status cs_attr_estimate_join(cs_attr *hs, int32_t u, int32_t v, void *stream, cs_estimate_t *out,
                                const cs_reps_t *reps)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    AttrHandle &h = hs->h;
    if (u < 0 || v < 0 || u >= h.g.n_attr || v >= h.g.n_attr || u == v)
        return fail(CS_EINVAL, "attributes out of range or equal");
    if (h.g.psi[u] != h.g.psi[v]) return fail(CS_EINVAL, "attributes of different components are not joined");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = (int)std::min<uint32_t>(kAttrDotBlocks, (h.m + kAttrBlock - 1) / kAttrBlock);
    const size_t bytes = (size_t)h.d * nb * sizeof(DotPartial);
    if (h.work_bytes < bytes) {
        CSK_HIP(hipStreamSynchronize(s));
        if (h.work) (void)hipFree(h.work);
        h.work = nullptr;
        h.work_bytes = 0;
        if (hipMalloc(&h.work, bytes) != hipSuccess) return fail(CS_ENOMEM, "attribute estimate partials");
        h.work_bytes = bytes;
    }
    if (h.host_bytes < bytes) {
        if (h.host) (void)hipHostFree(h.host);
        h.host = nullptr;
        h.host_bytes = 0;
        if (hipHostMalloc(&h.host, bytes, hipHostMallocDefault) != hipSuccess)
            return fail(CS_ENOMEM, "attribute estimate staging");
        h.host_bytes = bytes;
    }
    DotPartial *dp = static_cast<DotPartial *>(h.work);
    hipLaunchKernelGGL(k_attr_dot, dim3(nb, h.d), dim3(kAttrBlock), 0, s, h.counters + (size_t)u * h.d * h.m,
                       h.counters + (size_t)v * h.d * h.m, h.m, dp);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipMemcpyAsync(h.host, dp, bytes, hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    // The wrapping 128-bit sum is X_t exactly when sum_j |x_j y_j| < 2^126; its fp64
    // value is below the true sum by at most its roundings (the product, one per addition
    // on a term's path: the thread's terms, the block's 256 partials, the nb partials).
    const DotPartial *hp = static_cast<const DotPartial *>(h.host);
    const double unit_rnd = 0x1p-53;
    const double slack = 1.0 + (2.0 + (double)h.m + kAttrBlock + nb) * unit_rnd * 1.01;
    std::vector<__int128> x(h.d);
    std::vector<double> val(h.d);
    std::vector<int> ex(h.d);
    int all = 1;
    for (uint32_t t = 0; t < h.d; ++t) {
        unsigned __int128 tot = 0;
        double bound = 0.0, fsum = 0.0;
        for (int b = 0; b < nb; ++b) {
            const DotPartial &p = hp[(size_t)t * nb + b];
            tot += ((unsigned __int128)p.hi << 64) | p.lo;
            bound += p.abs_sum;
            fsum += p.sum;
        }
        x[t] = (__int128)tot;
        ex[t] = std::isfinite(bound) && bound * slack < 0x1p126;
        all &= ex[t];
        val[t] = ex[t] ? i128_to_double_attr(x[t]) : fsum;
        if (reps) {
            if (reps->value) reps->value[t] = val[t];
            if (reps->lo) reps->lo[t] = ex[t] ? (int64_t)(uint64_t)tot : 0;
            if (reps->hi) reps->hi[t] = ex[t] ? (int64_t)(uint64_t)(tot >> 64) : 0;
            if (reps->exact) reps->exact[t] = ex[t];
            if (reps->bound) reps->bound[t] = 0.0;
        }
    }
    // lower median (exact integers when every repetition is exact, else fp64 values),
    // ties by repetition index
    for (uint32_t t = 0; t < h.d; ++t) {
        uint32_t rank = 0;
        for (uint32_t i = 0; i < h.d; ++i) {
            const bool less = all ? x[i] < x[t] : val[i] < val[t];
            const bool same = all ? x[i] == x[t] : val[i] == val[t];
            rank += less || (same && i < t);
        }
        if (rank == (h.d - 1) / 2) {
            out->value = val[t];
            out->exact = all;
            out->fits_i64 = all && x[t] >= (__int128)INT64_MIN && x[t] <= (__int128)INT64_MAX;
            out->value_i64 = out->fits_i64 ? (int64_t)x[t] : 0;
            out->d = (int32_t)h.d;
            out->n_modular = 0;
        }
    }
    return CS_OK;
}

cs_status cs_attr_read(const cs_attr *hs, int32_t u, int64_t *host_out)
{
    if (!hs || !host_out) return fail(CS_EINVAL, "null argument");
    const AttrHandle &h = hs->h;
    if (u < 0 || u >= h.g.n_attr) return fail(CS_EINVAL, "attribute out of range");
    CSK_HIP(hipDeviceSynchronize());
    CSK_HIP(hipMemcpy(host_out, h.counters + (size_t)u * h.d * h.m, (size_t)h.d * h.m * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    return CS_OK;
}

cs_status cs_attr_coefficients(const cs_attr *hs, uint64_t *sign_out, uint64_t *bin_out)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    if (sign_out) std::memcpy(sign_out, hs->h.sign.data(), hs->h.sign.size() * sizeof(uint64_t));
    if (bin_out) std::memcpy(bin_out, hs->h.bin.data(), hs->h.bin.size() * sizeof(uint64_t));
    return CS_OK;
}

}  // extern "C"
