// Ingestion filters (Sec. 4.1 processes each query's filter predicates while tuples
// stream in): the tuples that satisfy a conjunction of range predicates on non-join
// columns are copied into a per-device buffer, wavefront by wavefront (ballot, one
// atomic reservation per wavefront), and only they are sketched.  The copy's order
// differs from the input's; the counters, integer sums, do not depend on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "csk_internal.h"

namespace csk {

namespace {

constexpr int kFilterBlock = 256;

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

__global__ __launch_bounds__(kFilterBlock) void k_filter(const uint32_t *__restrict__ keys, int n_cols,
                                                         const int64_t *__restrict__ weights, uint64_t n,
                                                         const uint32_t *__restrict__ attrs, int n_attrs,
                                                         FilterSpec f, uint32_t *okeys, int64_t *ow,
                                                         unsigned long long *count)
{
    const int lane = threadIdx.x & 63;
    // grid-stride over whole blocks, so every lane of a wavefront reaches the ballot
    for (uint64_t base = (uint64_t)blockIdx.x * kFilterBlock; base < n;
         base += (uint64_t)gridDim.x * kFilterBlock) {
        const uint64_t i = base + threadIdx.x;
        bool keep = i < n;
        if (keep) {
            for (int p = 0; p < f.n; ++p) {
                const uint32_t v = attrs[i * (uint64_t)n_attrs + f.col[p]];
                keep = keep && v >= f.lo[p] && v <= f.hi[p];
            }
        }
        const unsigned long long mask = __ballot(keep);
        const int cnt = __popcll(mask);
        unsigned long long at = 0;
        if (lane == 0 && cnt) at = atomicAdd(count, (unsigned long long)cnt);
        at = __shfl(at, 0, 64);
        if (keep) {
            const uint64_t o = at + (uint64_t)__popcll(mask & ((1ull << lane) - 1ull));
            for (int c = 0; c < n_cols; ++c) okeys[o * n_cols + c] = keys[i * n_cols + c];
            if (weights) ow[o] = weights[i];
        }
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
                        const uint32_t **keys_out, const int64_t **weights_out, uint64_t *kept)
{
    FilterBuf &B = fbuf_of(device);
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
    const uint64_t blocks = std::min<uint64_t>((n + kFilterBlock - 1) / kFilterBlock, 65536);
    hipLaunchKernelGGL(k_filter, dim3((unsigned)blocks), dim3(kFilterBlock), 0, s, keys, n_cols, weights, n, attrs,
                       n_attrs, f, okeys, ow, count);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipMemcpyAsync(B.host_count, count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    B.used = true;
    B.last_stream = s;
    *keys_out = okeys;
    *weights_out = ow;
    *kept = *B.host_count;
    return CS_OK;
}

}  // namespace csk
