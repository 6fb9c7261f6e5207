// Exact 16-bit LDS counters for updates whose every Delta is +1 or -1 (shared by the
// plain and the batched update kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace csk {

// 16-bit variant for Deltas +-1: two counters per 32-bit LDS word, each stored as
// value + 2^15, so a whole repetition of m <= 2^16 buckets fits 128 KB of LDS.  A half
// is in range while it lies in the window [0x4000, 0xBFFF] (2^15 - 2^14 to 2^15 + 2^14 - 1);
// a half found outside it hands +-2^14 to the int64 sketch (global atomic) and takes it
// off its 16-bit half by compare-and-swap, only while it is still outside, so value +
// spilled stays exact.  The kernels run at most 1024 threads per workgroup, each with at
// most eight adds whose result it has not checked yet, so a half stays within
// [0x2000, 0xDFFF] and never carries into its neighbour.
constexpr uint32_t kBias16 = 0x8000u, kSpill16 = 0x4000u;

// Word increment of Delta = -1 (neg) or +1 on the half at bit `shift` (0 or 16).
__device__ __forceinline__ uint32_t inc16(uint32_t neg, uint32_t shift)
{
    return neg ? (0xFFFFFFFFu << shift) : (1u << shift);
}

// The half an increment from inc16 adds to.
__device__ __forceinline__ uint32_t shift16(uint32_t inc) { return (inc & 0xFFFFu) ? 0u : 16u; }

// Whether a half of old + inc (the word right after this thread's add) lies outside the
// window.  Adding 0x4000 to a half maps the window onto [0x8000, 0xFFFF]: top bit set and
// no carry out of the half; below the window the top bit is clear, above it the half
// carries out.  The low half's carry can only disturb the high half's test when the low
// half is itself outside, so a half inside the window is never missed and a false alarm
// only costs spill16 one look at its half.
__device__ __forceinline__ bool out16(uint32_t old, uint32_t inc)
{
    return ((old + inc + 0x40004000u) & 0x80008000u) != 0x80008000u;
}

__device__ __forceinline__ void spill16(uint32_t *w, uint32_t shift, unsigned long long *g)
{
    for (;;) {
        const uint32_t old = *reinterpret_cast<volatile uint32_t *>(w);
        const uint32_t h = (old >> shift) & 0xFFFFu;
        uint32_t nw;
        unsigned long long amt;
        if (h >= kBias16 + kSpill16) {
            nw = old - (kSpill16 << shift);
            amt = (unsigned long long)kSpill16;
        } else if (h < kBias16 - kSpill16) {
            nw = old + (kSpill16 << shift);
            amt = (unsigned long long)0 - (unsigned long long)kSpill16;
        } else {
            return;
        }
        if (atomicCAS(w, old, nw) == old) atomicAdd(g, amt);
    }
}

}  // namespace csk
