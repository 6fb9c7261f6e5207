// Device-side polynomial hashing over the Mersenne prime field p = 2^61 - 1.
//
// The sign hashes are degree-3 polynomials (a 4-wise independent family) and the bin
// hashes degree-1 polynomials (2-wise independent), as the initialization paragraph
// of Sec. 3.2 requires; Sec. 4 evaluates them over a Mersenne prime field.  Keys are
// 32-bit, so one Horner step v*x + a multiplies a 61-bit value by a 32-bit key: two
// 32x32->64 multiplies, then the Mersenne fold 2^61 = 1 (mod p).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "csk_internal.h"

namespace csk {

constexpr uint64_t kHashP = (1ull << 61) - 1;

// One Horner step: returns r = v * x + a (mod p) in redundant form.
// Invariant: v < 2^63 and a < 2^61 give r < 2^61 + 2^34 + 8 + 2^61 < 2^63, so steps
// chain without an intermediate fold; hcanon() reduces the final value.
__device__ __forceinline__ uint64_t hstep(uint64_t v, uint32_t x, uint64_t a)
{
    const uint64_t lo = (uint64_t)(uint32_t)v * (uint64_t)x;  // < 2^64
    // v * x = t * 2^32 + (lo mod 2^32) with t = (v >> 32) * x + (lo >> 32) < 2^63 + 2^32
    const uint64_t t = (uint64_t)(uint32_t)(v >> 32) * (uint64_t)x + (lo >> 32);
    // (v * x mod 2^61) + (v * x >> 61) + a, using 2^61 = 1 (mod p): the low 61 bits are
    // the word pair (lo mod 2^32, t mod 2^29), built in the high half of lo's register
    // pair, so the sum is one 64-bit add (seven instructions a step).  The add is
    // written as the instruction itself: left to the compiler, it reassociates the three
    // terms into zero-extended 64-bit adds.
    const uint64_t low61 = ((uint64_t)((uint32_t)t & 0x1FFFFFFFu) << 32) | (uint32_t)lo;
    const uint64_t s = (t >> 29) + a;
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"(low61), "v"(s));
    return r;
}

// hstep on a value held as two 32-bit words.
struct HPair {
    uint32_t lo, hi;
};
__device__ __forceinline__ HPair hstep_p(HPair v, uint32_t x, uint64_t a)
{
    const uint64_t r = hstep(((uint64_t)v.hi << 32) | v.lo, x, a);
    return HPair{(uint32_t)r, (uint32_t)(r >> 32)};
}
__device__ __forceinline__ HPair hpair(uint64_t v) { return HPair{(uint32_t)v, (uint32_t)(v >> 32)}; }

// Canonical residue in [0, p) of a redundant value r < 2^63.
__device__ __forceinline__ uint64_t hcanon(uint64_t r)
{
    r = (r & kHashP) + (r >> 61);  // < 2^61 + 4
    return r >= kHashP ? r - kHashP : r;
}

// b0 + b1 x mod p (canonical)
__device__ __forceinline__ uint64_t hash_deg1(const uint64_t *b, uint32_t x)
{
    return hcanon(hstep(b[1], x, b[0]));
}

// a0 + a1 x + a2 x^2 + a3 x^3 mod p (canonical)
__device__ __forceinline__ uint64_t hash_deg3(const uint64_t *a, uint32_t x)
{
    return hcanon(hstep(hstep(hstep(a[3], x, a[2]), x, a[1]), x, a[0]));
}

// Bucket of a tuple: j = (sum of its columns' canonical bin values) mod m (the sum is
// below 8 * 2^61 < 2^64).  A power-of-two m keeps the low bits; any other m uses a
// Barrett reduction with mdiv = floor((2^64 - 1) / m), whose quotient estimate is at most
// two below the true one.
struct BinMod {
    uint32_t m;
    uint32_t pow2;
    uint64_t mdiv;
    __device__ __forceinline__ uint32_t reduce(uint64_t s) const
    {
        if (pow2) return (uint32_t)s & (m - 1);
        uint64_t r = s - __umul64hi(s, mdiv) * (uint64_t)m;
        if (r >= m) r -= m;
        if (r >= m) r -= m;
        return (uint32_t)r;
    }
};

// Per-relation hashing plan as the kernels read it: joins at each key column and the
// bucket reduction.
struct DevPlan {
    int32_t n_edges[kMaxCols];
    BinMod bm;
};

template <int NC>
__device__ __forceinline__ void load_keys(const uint32_t *__restrict__ keys, uint64_t i, bool vec2,
                                          uint32_t (&x)[NC])
{
    if constexpr (NC == 2) {
        if (vec2) {
            const uint2 v = reinterpret_cast<const uint2 *>(keys)[i];
            x[0] = v.x;
            x[1] = v.y;
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = keys[i * NC + c];
}

// Hash one tuple for one repetition; `cf` points at that repetition's coefficients
// (per column: b0, b1, then a0..a3 per join).  Returns the bucket j in [0, m) and the
// sign bit (1 = negative).
template <int NC>
__device__ __forceinline__ void hash_rep(const uint64_t *__restrict__ cf, const DevPlan &plan,
                                         const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg)
{
    uint64_t js = 0;
    neg = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        js += hash_deg1(cf, x[c]);
        cf += 2;
        const int ne = plan.n_edges[c];
        for (int e = 0; e < ne; ++e) {
            neg ^= (uint32_t)hash_deg3(cf, x[c]) & 1u;
            cf += 4;
        }
    }
    j = plan.bm.reduce(js);
}

// Bucket only (for segments holding a bucket range, where signs are needed only for
// tuples inside the range).
template <int NC>
__device__ __forceinline__ uint32_t hash_bin(const uint64_t *__restrict__ cf, const DevPlan &plan,
                                             const uint32_t (&x)[NC])
{
    uint64_t js = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        js += hash_deg1(cf, x[c]);
        cf += 2 + 4 * plan.n_edges[c];
    }
    return plan.bm.reduce(js);
}

template <int NC>
__device__ __forceinline__ uint32_t hash_neg(const uint64_t *__restrict__ cf, const DevPlan &plan,
                                             const uint32_t (&x)[NC])
{
    uint32_t neg = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        cf += 2;
        for (int e = 0; e < plan.n_edges[c]; ++e) {
            neg ^= (uint32_t)hash_deg3(cf, x[c]) & 1u;
            cf += 4;
        }
    }
    return neg;
}

// (tuple chunk, segment) of a two-dimensional launch's workgroup.  Workgroups go to the 8 XCDs
// round-robin by linear id; the ids one XCD receives are given a contiguous run of the
// chunk-major order, so the segments of one tuple chunk run on one XCD (two at a run's
// ends) and that XCD's L2 fetches the chunk's keys once.
struct SegTile {
    uint32_t chunk, seg;
};
__device__ __forceinline__ SegTile seg_tile()
{
    const uint32_t G = gridDim.x * gridDim.y;
    const uint32_t L = blockIdx.x + blockIdx.y * gridDim.x;
    const uint32_t xcd = L & 7u, w = L >> 3;
    const uint32_t P = xcd * (G >> 3) + min(xcd, G & 7u) + w;  // a bijection of [0, G)
    return {P / gridDim.y, P % gridDim.y};
}

__host__ __device__ inline BinMod make_binmod(uint32_t m)
{
    BinMod b;
    b.m = m;
    b.pow2 = (m & (m - 1)) == 0 ? 1u : 0u;
    b.mdiv = ~0ull / m;
    return b;
}

// Coefficients of one repetition for relations whose every key column takes part in
// exactly one join (chains, stars): b0, b1, a0..a3 per column, held in registers.
template <int NC>
struct CoefE1 {
    uint64_t b0[NC], b1[NC], a[NC][4];
    template <typename P>  // a generic, global or constant address-space pointer
    __device__ __forceinline__ void load(P cf)
    {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            b0[c] = cf[6 * c];
            b1[c] = cf[6 * c + 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) a[c][k] = cf[6 * c + 2 + k];
        }
    }
    __device__ __forceinline__ uint32_t bin(const uint32_t (&x)[NC]) const
    {
        uint32_t j = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) j += (uint32_t)hcanon(hstep(b1[c], x[c], b0[c]));
        return j;
    }
    __device__ __forceinline__ uint32_t neg(const uint32_t (&x)[NC]) const
    {
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            s ^= (uint32_t)hcanon(hstep(hstep(hstep(a[c][3], x[c], a[c][2]), x[c], a[c][1]), x[c], a[c][0])) & 1u;
        return s;
    }
    // bin() and neg() without the canonical reduction, for the common case.  A Horner
    // result r < 2^63 is r = q 2^61 + u (q = r >> 61, u < 2^61), and r mod p = q + u -
    // p [q + u >= p].  The bins need r mod p only modulo 2^32 and the signs only its
    // parity; p = -1 (mod 2^32) and p is odd, so r mod p = r_lo + q + c (mod 2^32) and
    // its parity is (r_lo ^ q ^ c) & 1, with c = [q + u >= p].  c can be 1 only when the
    // top 29 bits of u are all ones (u >= p - 3); `flag` is the largest (r_hi | 0xE0000000)
    // over the tuple's hashes, and a caller that finds flag >= 0xFFFFFFFF takes bin() and
    // neg() instead (about once in 2^29 hashes).
    __device__ __forceinline__ void bin_neg_fast(const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg,
                                                 uint32_t &flag) const
    {
        j = 0;
        neg = 0;
        flag = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const HPair rb = hstep_p(hpair(b1[c]), x[c], b0[c]);
            j += rb.lo + (rb.hi >> 29);
            const HPair rs = hstep_p(hstep_p(hstep_p(hpair(a[c][3]), x[c], a[c][2]), x[c], a[c][1]), x[c], a[c][0]);
            neg ^= rs.lo ^ (rs.hi >> 29);
            flag = max(flag, max(rb.hi | 0xE0000000u, rs.hi | 0xE0000000u));
        }
        neg &= 1u;
    }
};

}  // namespace csk
