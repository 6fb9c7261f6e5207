// Ingestion filters (Sec. 4.1 processes each query's filter predicates while tuples
// stream in): the tuples that satisfy a conjunction of range predicates on non-join
// columns are copied into a per-device buffer, tile by tile (one atomic reservation per
// tile of 4096 tuples), and only they are sketched.  The copy's order
// differs from the input's; the counters, integer sums, do not depend on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>

#include "csk_internal.h"

namespace csk {

namespace {

constexpr int kFilterBlock = 256;

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// A workgroup takes a tile of kFilterBlock x kFilterPer tuples (a thread's tuples are
// kFilterBlock apart, so every load is coalesced), counts the tuples each thread keeps,
// scans the counts in LDS, reserves the tile's slots with one atomic, and writes.
constexpr int kFilterPer = 16;

__global__ __launch_bounds__(kFilterBlock) void k_filter(const uint32_t *__restrict__ keys, int n_cols,
                                                         const int64_t *__restrict__ weights, uint64_t n,
                                                         const uint32_t *__restrict__ attrs, int n_attrs,
                                                         FilterSpec f, uint32_t *okeys, int64_t *ow,
                                                         unsigned long long *count)
{
    __shared__ uint32_t s_cnt[kFilterBlock];
    __shared__ unsigned long long s_base;
    const uint64_t tile = (uint64_t)kFilterBlock * kFilterPer;
    for (uint64_t t0 = (uint64_t)blockIdx.x * tile; t0 < n; t0 += (uint64_t)gridDim.x * tile) {
        uint32_t keep = 0;  // bit u: tuple t0 + u * kFilterBlock + threadIdx.x passes
#pragma unroll
        for (int u = 0; u < kFilterPer; ++u) {
            const uint64_t i = t0 + (uint64_t)u * kFilterBlock + threadIdx.x;
            bool k = i < n;
            if (k)
                for (int p = 0; p < f.n; ++p) {
                    const uint32_t v = attrs[i * (uint64_t)n_attrs + f.col[p]];
                    k = k && v >= f.lo[p] && v <= f.hi[p];
                }
            keep |= (uint32_t)k << u;
        }
        const uint32_t mine = __popc(keep);
        s_cnt[threadIdx.x] = mine;
        __syncthreads();
        // inclusive scan of the per-thread counts (Hillis-Steele in LDS)
        for (int off = 1; off < kFilterBlock; off <<= 1) {
            const uint32_t add = threadIdx.x >= (unsigned)off ? s_cnt[threadIdx.x - off] : 0u;
            __syncthreads();
            s_cnt[threadIdx.x] += add;
            __syncthreads();
        }
        if (threadIdx.x == kFilterBlock - 1)
            s_base = s_cnt[threadIdx.x] ? atomicAdd(count, (unsigned long long)s_cnt[threadIdx.x]) : 0ull;
        __syncthreads();
        uint64_t o = s_base + s_cnt[threadIdx.x] - mine;
        for (int u = 0; u < kFilterPer; ++u) {
            if (!((keep >> u) & 1u)) continue;
            const uint64_t i = t0 + (uint64_t)u * kFilterBlock + threadIdx.x;
            for (int c = 0; c < n_cols; ++c) okeys[o * n_cols + c] = keys[i * n_cols + c];
            if (weights) ow[o] = weights[i];
            ++o;
        }
        __syncthreads();  // s_cnt and s_base are rewritten by the next tile
    }
}

struct FilterBuf {
    std::mutex mu;
    void *buf = nullptr;
    size_t bytes = 0;
    unsigned long long *host_count = nullptr;  // pinned
    hipStream_t last_stream = nullptr;
    bool used = false;
};
std::mutex g_fmu;
std::map<int, FilterBuf *> g_fbufs;

FilterBuf &fbuf_of(int device)
{
    std::lock_guard<std::mutex> lk(g_fmu);
    FilterBuf *&b = g_fbufs[device];
    if (!b) b = new FilterBuf();
    return *b;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

cs_status filter_tuples(int device, const uint32_t *keys, int n_cols, const int64_t *weights, uint64_t n,
                        const uint32_t *attrs, int n_attrs, const FilterSpec &f, hipStream_t s,
                        const std::function<cs_status(const uint32_t *, const int64_t *, uint64_t)> &consume)
{
    FilterBuf &B = fbuf_of(device);
    // held until `consume` has enqueued its reads of the buffer: another caller on this
    // device cannot overwrite or reallocate the buffer in between
    std::lock_guard<std::mutex> lk(B.mu);
    // the buffer's last reader (an update on another stream) must have finished
    if (B.used && s != B.last_stream) CSK_HIP(hipDeviceSynchronize());
    const size_t o_keys = 256;
    const size_t o_w = o_keys + align256(n * (size_t)n_cols * sizeof(uint32_t));
    const size_t need = o_w + (weights ? align256(n * sizeof(int64_t)) : 0);
    if (B.bytes < need) {
        CSK_HIP(hipStreamSynchronize(s));
        if (B.buf) hipFree(B.buf);
        B.buf = nullptr;
        B.bytes = 0;
        if (hipMalloc(&B.buf, need) != hipSuccess) return fail(CS_ENOMEM, "filter buffer");
        B.bytes = need;
    }
    if (!B.host_count && hipHostMalloc(reinterpret_cast<void **>(&B.host_count), sizeof(unsigned long long),
                                       hipHostMallocDefault) != hipSuccess)
        return fail(CS_ENOMEM, "filter count staging");
    char *base = static_cast<char *>(B.buf);
    unsigned long long *count = reinterpret_cast<unsigned long long *>(base);
    uint32_t *okeys = reinterpret_cast<uint32_t *>(base + o_keys);
    int64_t *ow = weights ? reinterpret_cast<int64_t *>(base + o_w) : nullptr;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, count);
    CSK_HIP(hipGetLastError());
    const uint64_t tile = (uint64_t)kFilterBlock * kFilterPer;
    const uint64_t blocks = std::min<uint64_t>((n + tile - 1) / tile, 8192);
    hipLaunchKernelGGL(k_filter, dim3((unsigned)blocks), dim3(kFilterBlock), 0, s, keys, n_cols, weights, n, attrs,
                       n_attrs, f, okeys, ow, count);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipMemcpyAsync(B.host_count, count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    B.used = true;
    B.last_stream = s;
    return consume(okeys, ow, (uint64_t)*B.host_count);
}

}  // namespace csk
