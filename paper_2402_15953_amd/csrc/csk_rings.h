// Arithmetic used by the transforms: complex fp64 (the FFT of Alg. 3) and Montgomery
// arithmetic modulo 31-bit NTT primes (the exact modular evaluation).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace csk {

struct RingC {
    using T = double2;
    __device__ __forceinline__ T add(T a, T b) const { return make_double2(a.x + b.x, a.y + b.y); }
    __device__ __forceinline__ T sub(T a, T b) const { return make_double2(a.x - b.x, a.y - b.y); }
    __device__ __forceinline__ T mul(T a, T w) const
    {
        return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
    }
};

struct RingM {
    using T = uint32_t;
    uint32_t p;
    uint32_t pinv_neg;  // -p^{-1} mod 2^32
    __device__ __forceinline__ T add(T a, T b) const
    {
        const uint32_t s = a + b;
        return s >= p ? s - p : s;
    }
    __device__ __forceinline__ T sub(T a, T b) const { return a >= b ? a - b : a + p - b; }
    // Montgomery product a * w * 2^-32 mod p; needs a * w < p * 2^32.
    __device__ __forceinline__ T mul(T a, T w) const
    {
        const uint64_t t = (uint64_t)a * w;
        const uint32_t q = (uint32_t)t * pinv_neg;
        const uint32_t u = (uint32_t)((t + (uint64_t)q * p) >> 32);  // < 2p
        return min(u, u - p);  // u - p wraps above u when u < p
    }
};

// Montgomery form of an int64 value modulo p (r2 = 2^64 mod p, r3 = 2^96 mod p,
// neg2_64 = Montgomery form of -2^64).
__device__ __forceinline__ uint32_t mont_from_i64(const RingM &R, int64_t c, uint32_t r2, uint32_t r3,
                                                  uint32_t neg2_64)
{
    const uint64_t u = (uint64_t)c;
    uint32_t s = R.add(R.mul((uint32_t)(u >> 32), r3), R.mul((uint32_t)u, r2));
    if (c < 0) s = R.add(s, neg2_64);
    return s;
}

}  // namespace csk
