// Exact 16-bit LDS counters for updates whose every Delta is +1 or -1 (shared by the
// plain and the batched update kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace csk {

// 16-bit variant for Deltas +-1: two counters per 32-bit LDS word, each stored as
// value + 2^15, so a whole repetition of m <= 2^16 buckets fits 128 KB of LDS.  A
// counter that reaches 2^15 +- 2^14 hands 2^14 to the int64 sketch (global atomic) and
// takes it off its 16-bit half by compare-and-swap, only while it is still beyond the
// threshold; a half therefore stays within 2^15 +- (2^14 + in-flight adds) and never
// carries into its neighbour, and value + spilled stays exact.  The kernels run at most
// 1024 threads per workgroup, each with at most two adds whose returned value it has
// not checked yet, so a half stays within [0x3800, 0xC800].
constexpr uint32_t kBias16 = 0x8000u, kHi16 = 0xC000u, kLo16 = 0x4000u, kSpill16 = 0x4000u;

__device__ __forceinline__ void spill16(uint32_t *w, uint32_t shift, unsigned long long *g)
{
    for (;;) {
        const uint32_t old = *reinterpret_cast<volatile uint32_t *>(w);
        const uint32_t h = (old >> shift) & 0xFFFFu;
        uint32_t nw;
        unsigned long long amt;
        if (h >= kHi16) {
            nw = old - (kSpill16 << shift);
            amt = (unsigned long long)kSpill16;
        } else if (h <= kLo16) {
            nw = old + (kSpill16 << shift);
            amt = (unsigned long long)0 - (unsigned long long)kSpill16;
        } else {
            return;
        }
        if (atomicCAS(w, old, nw) == old) atomicAdd(g, amt);
    }
}

}  // namespace csk
