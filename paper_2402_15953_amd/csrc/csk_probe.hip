// Machine-balance probes of the update's two rooflines, measured on the device the
// library runs on: the rate of the Horner step (v <- v * x + a mod 2^61 - 1 with a
// 32-bit x, the update's unit of work, Alg. 2's hashes) when nothing else limits it,
// and the rate at which a kernel streams a large buffer from HBM (the key stream's
// bound).  The update and estimate kernels are measured against these two figures.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "csk_hash.h"
#include "csk_internal.h"

namespace csk {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;  // independent Horner chains per lane

// Every lane runs kProbeChains independent chains of `iters` steps each, with keys that
// differ per lane and chain; the chains' final values are folded into one word per
// lane so that no step is dead code.
__global__ __launch_bounds__(kProbeBlock) void k_probe_horner(uint64_t iters, uint64_t a, uint64_t *out)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t v[kProbeChains];
    uint32_t x[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
        v[c] = (a + gid * 0x9E3779B9ull + c) & kHashP;
        x[c] = gid * 2654435761u + (uint32_t)c * 40503u;
    }
    for (uint64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) v[c] = hstep(v[c], x[c], a);
    }
    uint64_t f = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) f ^= v[c];
    out[gid] = f;
}

// Grid-stride read of `words` 16-byte words, four independent loads in flight per lane,
// xor-folded into one word per lane.
__global__ __launch_bounds__(kProbeBlock) void k_probe_read(const uint4 *__restrict__ p, uint64_t words,
                                                            uint32_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (; i + 3 * stride < words; i += 4 * stride) {
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < words; i += stride) {
        const uint4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace
}  // namespace csk

extern "C" {

cs_status cs_k0_horner(uint64_t iters, double *steps_per_s)
{
    using namespace csk;
    if (!steps_per_s || iters == 0) return fail(CS_EINVAL, "null output or zero iterations");
    int dev = 0, n_cu = 256;
    CSK_HIP(hipGetDevice(&dev));
    CSK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint32_t blocks = (uint32_t)n_cu * 16;  // 16 waves per CU: 4 per SIMD
    uint64_t *out = nullptr;
    CSK_HIP(hipMalloc(&out, (size_t)blocks * kProbeBlock * sizeof(uint64_t)));
    hipEvent_t e0, e1;
    CSK_HIP(hipEventCreate(&e0));
    CSK_HIP(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_probe_horner, dim3(blocks), dim3(kProbeBlock), 0, nullptr, iters / 8 + 1, 12345ull, out);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipEventRecord(e0, nullptr));
    hipLaunchKernelGGL(k_probe_horner, dim3(blocks), dim3(kProbeBlock), 0, nullptr, iters, 67890ull, out);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipEventRecord(e1, nullptr));
    CSK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    CSK_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    *steps_per_s = (double)blocks * kProbeBlock * kProbeChains * (double)iters / (ms * 1e-3);
    return CS_OK;
}

cs_status cs_k0_stream_read(const void *buf, uint64_t bytes, int32_t passes, double *bytes_per_s)
{
    using namespace csk;
    if (!buf || !bytes_per_s || bytes < 16 || passes < 1) return fail(CS_EINVAL, "bad probe arguments");
    int dev = 0, n_cu = 256;
    CSK_HIP(hipGetDevice(&dev));
    CSK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    cs_status chk = check_device_array(buf, bytes, dev, "probe buffer");
    if (chk != CS_OK) return chk;
    const uint64_t words = bytes / 16;
    const uint32_t blocks = (uint32_t)n_cu * 8;
    uint32_t *out = nullptr;
    CSK_HIP(hipMalloc(&out, (size_t)blocks * kProbeBlock * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CSK_HIP(hipEventCreate(&e0));
    CSK_HIP(hipEventCreate(&e1));
    const uint4 *p = static_cast<const uint4 *>(buf);
    hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(kProbeBlock), 0, nullptr, p, words, out);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipEventRecord(e0, nullptr));
    for (int i = 0; i < passes; ++i)
        hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(kProbeBlock), 0, nullptr, p, words, out);
    CSK_HIP(hipGetLastError());
    CSK_HIP(hipEventRecord(e1, nullptr));
    CSK_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    CSK_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    *bytes_per_s = (double)words * 16.0 * passes / (ms * 1e-3);
    return CS_OK;
}

}  // extern "C"
