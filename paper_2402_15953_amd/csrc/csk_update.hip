// Sketch update kernels (Alg. 2; Eq. 2-4), one launch per call for one relation.
//
// Per tuple and repetition t: bin j = (sum over key columns of the component's bin
// hash) mod m; sign = product over key columns of the sign hashes of every join at
// that column; counter c[t][j] += sign * Delta.  Counters are int64 and adds wrap, so
// any order of the atomic adds gives the same bits.
//
// Strategies:
//   global atomic  - grid-stride over tuples, one device-scope int64 atomic per
//                    (tuple, repetition); the key stream is read once, coalesced.
//   LDS segmented  - the [d][m] counters are cut into segments that fit one CU's LDS;
//                    workgroup (chunk, segment) accumulates its chunk's tuples that land
//                    in its segment with LDS atomics, stores the partial sums, and a
//                    reduce kernel adds them into the sketch.  Replaces global atomics
//                    (about 2.4e10/s for the whole chip) by LDS atomics.
//   wave aggregate - global atomic, but lanes of a wavefront that hit the same
//                    counter first combine their values through LDS, so a hot bucket
//                    costs one atomic per wavefront instead of one per lane.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <map>
#include <mutex>

#include "csk_counters16.h"
#include "csk_handle.h"
#include "csk_hash.h"
#include "csk_internal.h"

namespace csk {

namespace {

constexpr int kBlock = 256;
constexpr int kSegBlock = 1024;
constexpr uint32_t kSeg16Words = 1u << 15;  // 128 KB: 2^16 16-bit counters
constexpr int kSeg16Group = 4;              // tuples hashed together by one thread

template <int NC>
__global__ __launch_bounds__(kBlock) void k_update_global(const uint32_t *__restrict__ keys,
                                                          const int64_t *__restrict__ weights,
                                                          uint64_t n, const uint64_t *__restrict__ coef,
                                                          int32_t cpr, unsigned long long *sketch,
                                                          uint32_t m, int32_t d, DevPlan plan, bool vec2)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        uint32_t x[NC];
        load_keys<NC>(keys, i, vec2, x);
        const int64_t delta = weights ? weights[i] : 1;
        const uint64_t *cf = coef;
        for (int t = 0; t < d; ++t, cf += cpr) {
            uint32_t j, neg;
            hash_rep<NC>(cf, plan, x, j, neg);
            const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
            atomicAdd(sketch + (size_t)t * m + j, (unsigned long long)val);
        }
    }
}

// ---------------------------------------------------------------- ingestion filters
//
// Sec. 4.1 applies each query's filter predicates while its relations stream in: only
// the tuples whose attribute columns pass every predicate reach the sketch.  The
// filtered kernels evaluate the predicates on attrs [n][n_attrs] (tuple-major uint32)
// themselves and hash only the tuples that pass; the sketch is that of the kept tuples.

// Whether tuple i passes every predicate of f (lo <= attrs[i][col] <= hi).
__device__ __forceinline__ bool passes(const uint32_t *__restrict__ attrs, int n_attrs, uint64_t i,
                                       const FilterSpec &f)
{
    bool k = true;
    for (int p = 0; p < f.n; ++p) {
        const uint32_t v = attrs[i * (uint64_t)n_attrs + f.col[p]];
        k = k && v >= f.lo[p] && v <= f.hi[p];
    }
    return k;
}

// Global-atomic update of the kept tuples (every shape of relation, any weights).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_update_global_f(const uint32_t *__restrict__ keys,
                                                            const int64_t *__restrict__ weights, uint64_t n,
                                                            const uint64_t *__restrict__ coef, int32_t cpr,
                                                            unsigned long long *sketch, uint32_t m, int32_t d,
                                                            DevPlan plan, bool vec2,
                                                            const uint32_t *__restrict__ attrs, int32_t n_attrs,
                                                            FilterSpec f, unsigned long long *kept)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t mine = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        if (!passes(attrs, n_attrs, i, f)) continue;
        ++mine;
        uint32_t x[NC];
        load_keys<NC>(keys, i, vec2, x);
        const int64_t delta = weights ? weights[i] : 1;
        const uint64_t *cf = coef;
        for (int t = 0; t < d; ++t, cf += cpr) {
            uint32_t j, neg;
            hash_rep<NC>(cf, plan, x, j, neg);
            const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
            atomicAdd(sketch + (size_t)t * m + j, (unsigned long long)val);
        }
    }
    if (kept) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
        if ((threadIdx.x & 63) == 0 && mine) atomicAdd(kept, (unsigned long long)mine);
    }
}

// Wave-aggregated variant: per repetition, every lane writes its (bucket, value) into a
// per-wave LDS slot; lanes then find the first lane of the wave with the same bucket
// (a scan over the wave's 64 slots, LDS broadcast reads); the first lane sums the
// values of all its duplicates and issues the only atomic.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_update_waveagg(const uint32_t *__restrict__ keys,
                                                           const int64_t *__restrict__ weights,
                                                           uint64_t n, const uint64_t *__restrict__ coef,
                                                           int32_t cpr, unsigned long long *sketch,
                                                           uint32_t m, int32_t d, DevPlan plan, bool vec2)
{
    __shared__ uint32_t s_bin[kBlock];
    __shared__ uint64_t s_val[kBlock];
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    // every thread of the block runs the same number of iterations (uniform loop bound)
    const uint64_t iters = (n + stride - 1) / stride;
    for (uint64_t it = 0; it < iters; ++it) {
        const uint64_t i = it * stride + (uint64_t)blockIdx.x * kBlock + threadIdx.x;
        const bool valid = i < n;
        uint32_t x[NC];
        int64_t delta = 0;
        if (valid) {
            load_keys<NC>(keys, i, vec2, x);
            delta = weights ? weights[i] : 1;
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = 0;
        }
        const uint64_t *cf = coef;
        for (int t = 0; t < d; ++t, cf += cpr) {
            uint32_t j, neg;
            hash_rep<NC>(cf, plan, x, j, neg);
            const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
            const uint32_t key = valid ? j : 0xFFFFFFFFu;
            s_bin[threadIdx.x] = key;
            s_val[threadIdx.x] = val;
            __syncthreads();
            int first = lane;
            for (int l = 0; l < lane; ++l) {
                if (s_bin[wbase + l] == key) {
                    first = l;
                    break;
                }
            }
            if (valid && first == lane) {
                uint64_t sum = val;
                for (int l = lane + 1; l < 64; ++l)
                    if (s_bin[wbase + l] == key) sum += s_val[wbase + l];
                if (sum) atomicAdd(sketch + (size_t)t * m + j, (unsigned long long)sum);
            }
            __syncthreads();
        }
    }
}

// LDS-segmented variant.  The flattened counter space [d][m] is cut into segments of
// R cells; block (c, s) accumulates the tuples of chunk c that land in segment s into
// LDS counters (int32 when every Delta is +1, else int64), then stores them as the
// chunk's partial sums; k_seg_reduce adds the partials of all chunks into the sketch.
// A segment holds whole repetitions when m <= R, else a bucket range of one
// repetition (its tuples' signs are then only needed for in-range buckets).

template <int NC, typename CT, bool E1>
__global__ __launch_bounds__(kSegBlock) void k_update_seg(const uint32_t *__restrict__ keys,
                                                          const int64_t *__restrict__ weights, uint64_t n,
                                                          const uint64_t *__restrict__ coef, int32_t cpr,
                                                          DevPlan plan, uint32_t m, int32_t log2m, int32_t d,
                                                          uint32_t R, uint64_t chunk, bool vec2, CT *partial)
{
    extern __shared__ __align__(16) unsigned char s_raw[];
    CT *s_c = reinterpret_cast<CT *>(s_raw);
    const uint64_t cells = (uint64_t)d * m;
    const SegTile wg = seg_tile();
    const uint64_t cell0 = (uint64_t)wg.seg * R;
    const uint64_t cell1 = cell0 + R < cells ? cell0 + R : cells;
    const uint32_t span = (uint32_t)(cell1 - cell0);
    const int t0 = (int)(cell0 / m);
    const int t1 = (int)((cell1 - 1) / m);
    const bool whole = R >= m;
    for (uint32_t e = threadIdx.x; e < span; e += kSegBlock) s_c[e] = 0;
    __syncthreads();
    const uint64_t begin = (uint64_t)wg.chunk * chunk;
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    // repetition outermost: its coefficients stay in scalar registers over the tuples
    for (int t = t0; t <= t1; ++t) {
        const uint64_t *cf = coef + (size_t)t * cpr;
        CoefE1<NC> K;
        if constexpr (E1) K.load(cf);
        const uint32_t row = (uint32_t)((uint64_t)t * m - cell0);  // may wrap; used mod 2^32
        for (uint64_t i = begin + threadIdx.x; i < end; i += kSegBlock) {
            uint32_t x[NC];
            load_keys<NC>(keys, i, vec2, x);
            uint32_t j, neg;
            if constexpr (E1) {  // power-of-two m only
                j = K.bin(x) & (m - 1);
                const uint32_t loc = row + j;
                if (!whole && loc >= span) continue;  // bucket outside this segment
                neg = K.neg(x);
            } else if (whole) {
                hash_rep<NC>(cf, plan, x, j, neg);
            } else {
                // bins first; signs only for buckets inside this segment
                j = hash_bin<NC>(cf, plan, x);
                if (row + j >= span) continue;
                neg = hash_neg<NC>(cf, plan, x);
            }
            const uint32_t loc = row + j;
            const int64_t delta = weights ? weights[i] : 1;
            if constexpr (sizeof(CT) == 4) {
                const int32_t v32 = (int32_t)delta;  // +1, or +-1 with unit weights
                atomicAdd(&s_c[loc], neg ? -v32 : v32);
            } else {
                const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_c[loc]), (unsigned long long)val);
            }
        }
    }
    __syncthreads();
    CT *out = partial + (size_t)wg.chunk * cells + cell0;
    for (uint32_t e = threadIdx.x; e < span; e += kSegBlock) out[e] = s_c[e];
}

// Compacting variant for segments that hold a bucket range of one repetition (m > R),
// one join per key column, Deltas +-1 (int32 counters).  Each wavefront hashes the bins
// of 64 tuples, appends the in-range ones (keys, counter offset, sign of Delta) to its
// LDS queue, and computes the sign hashes only when 64 are queued, so sign work is done
// at full SIMD width instead of once per range.
constexpr int kQCap = 128;  // queue entries per wavefront (< 64 pending + 64 pushed)

template <int NC>
__global__ __launch_bounds__(kSegBlock) void k_update_seg_compact(const uint32_t *__restrict__ keys,
                                                                  const int64_t *__restrict__ weights,
                                                                  uint64_t n, const uint64_t *__restrict__ coef,
                                                                  int32_t cpr, uint32_t m, int32_t log2m,
                                                                  int32_t d, uint32_t R, uint64_t chunk, bool vec2,
                                                                  int32_t *partial)
{
    extern __shared__ __align__(16) unsigned char s_raw[];
    int32_t *s_c = reinterpret_cast<int32_t *>(s_raw);                                // [R]
    uint32_t *q_x = reinterpret_cast<uint32_t *>(s_raw + (size_t)R * sizeof(int32_t));  // [waves][NC][kQCap]
    uint32_t *q_l = q_x + (kSegBlock / 64) * NC * kQCap;                              // [waves][kQCap]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t *qx = q_x + wave * NC * kQCap;
    uint32_t *ql = q_l + wave * kQCap;
    const uint64_t cells = (uint64_t)d << log2m;
    const SegTile wg = seg_tile();
    const uint64_t cell0 = (uint64_t)wg.seg * R;
    const int t = (int)(cell0 >> log2m);
    const uint32_t off = (uint32_t)(cell0 - ((uint64_t)t << log2m));  // first bucket of the range
    for (uint32_t e = threadIdx.x; e < R; e += kSegBlock) s_c[e] = 0;
    __syncthreads();
    CoefE1<NC> K;
    K.load(coef + (size_t)t * cpr);
    const uint64_t begin = (uint64_t)wg.chunk * chunk;
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    uint32_t head = 0, count = 0;  // wave-uniform queue state
    auto drain = [&](uint32_t k) {  // lanes < k take one queued entry each
        if ((uint32_t)lane < k) {
            const uint32_t slot = (head + lane) & (kQCap - 1);
            uint32_t x[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = qx[c * kQCap + slot];
            const uint32_t l = ql[slot];
            const int32_t v = (K.neg(x) ^ (l >> 31)) ? -1 : 1;
            atomicAdd(&s_c[l & 0x7FFFFFFFu], v);
        }
        head = (head + k) & (kQCap - 1);
        count -= k;
    };
    for (uint64_t base = begin + (uint64_t)wave * 64; base < end; base += kSegBlock) {
        const uint64_t i = base + lane;
        bool in = false;
        uint32_t x[NC], loc = 0;
        if (i < end) {
            load_keys<NC>(keys, i, vec2, x);
            const uint32_t j = (K.bin(x) & (m - 1)) - off;
            if (j < R) {
                in = true;
                loc = j | ((weights && weights[i] < 0) ? 0x80000000u : 0u);
            }
        }
        const uint64_t mask = __ballot(in);
        if (in) {
            const uint32_t pos = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            const uint32_t slot = (head + count + pos) & (kQCap - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) qx[c * kQCap + slot] = x[c];
            ql[slot] = loc;
        }
        count += (uint32_t)__popcll(mask);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (count >= 64) drain(64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (count > 0) drain(count);
    __syncthreads();
    int32_t *out = partial + (size_t)wg.chunk * cells + cell0;
    for (uint32_t e = threadIdx.x; e < R; e += kSegBlock) out[e] = s_c[e];
}

template <int NC, bool E1, bool HW>
__global__ __launch_bounds__(kSegBlock) void k_update_seg16(const uint32_t *__restrict__ keys,
                                                            const int64_t *__restrict__ weights, uint64_t n,
                                                            const uint64_t *__restrict__ coef, int32_t cpr,
                                                            DevPlan plan, uint32_t m, int32_t log2m, int32_t d,
                                                            uint32_t R, uint64_t chunk, bool vec2,
                                                            uint32_t *partial, unsigned long long *sketch,
                                                            uint32_t canon_thresh)
{
    // [R / 2] words, two counters each (R <= 2^16); a fixed array, so that its LDS
    // address is a constant the compiler folds into the address arithmetic
    __shared__ uint32_t s_w[kSeg16Words];
    const uint64_t cells = (uint64_t)d * m;
    const SegTile wg = seg_tile();
    const uint64_t cell0 = (uint64_t)wg.seg * R;
    const uint64_t cell1 = cell0 + R < cells ? cell0 + R : cells;
    const uint32_t span = (uint32_t)(cell1 - cell0);  // even: R is even (so is cells)
    const int t0 = (int)(cell0 / m);
    const int t1 = (int)((cell1 - 1) / m);
    for (uint32_t e = threadIdx.x; e < span / 2; e += kSegBlock) s_w[e] = (kBias16 << 16) | kBias16;
    __syncthreads();
    const uint64_t begin = (uint64_t)wg.chunk * chunk;
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    for (int t = t0; t <= t1; ++t) {
        const uint64_t *cf = coef + (size_t)t * cpr;
        CoefE1<NC> K;
        if constexpr (E1) K.load(cf);
        const uint32_t row = (uint32_t)((uint64_t)t * m - cell0);
        unsigned long long *srow = sketch + (uint64_t)t * m;
        // Tuples go in groups of kSeg16Group: all are hashed in one straight-line block
        // (independent chains for the scheduler, one test of the rare full-reduction
        // flag), their LDS adds are issued, and only then are the words the previous
        // group's adds returned checked; the next group's keys are in flight meanwhile.
        // Neither the LDS latency nor the loads stall the wavefront.  A thread has at most
        // 2 * kSeg16Group adds whose result it has not checked: with 1024 threads a half
        // stays within 2^15 +- (2^14 + 8 * 1024).
        constexpr int G = kSeg16Group;
        struct Pend {
            uint32_t old, inc, j;  // word before the add, the increment, the bucket
            uint32_t *w;
        };
        Pend pend[G];
#pragma unroll
        for (int g = 0; g < G; ++g) pend[g] = Pend{kBias16 * 0x10001u, 0u, 0u, s_w};  // in range
        auto check = [&]() {
            bool any = false;
#pragma unroll
            for (int g = 0; g < G; ++g) any |= out16(pend[g].old, pend[g].inc);
            if (any) {
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (out16(pend[g].old, pend[g].inc))
                        spill16(pend[g].w, shift16(pend[g].inc), srow + pend[g].j);
            }
        };
        auto hash1 = [&](const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg, uint32_t &flag) {
            if constexpr (E1) {
                K.bin_neg_fast(x, j, neg, flag);
            } else {
                hash_rep<NC>(cf, plan, x, j, neg);
                flag = 0;
            }
        };
        auto exact1 = [&](const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg) {
            if constexpr (E1) {
                j = K.bin(x);
                neg = K.neg(x);
            }
        };
        auto add1 = [&](uint32_t j, uint32_t neg, int64_t wt) -> Pend {
            if constexpr (E1) j &= m - 1;
            if constexpr (HW) neg ^= (uint32_t)((uint64_t)wt >> 63);
            const uint32_t loc = row + j;
            uint32_t *w = &s_w[loc >> 1];
            const uint32_t inc = inc16(neg, (loc & 1u) << 4);
            return Pend{atomicAdd(w, inc), inc, j, w};
        };
        auto load = [&](uint64_t k, uint32_t (&x)[NC], int64_t &wt) {
            load_keys<NC>(keys, k, vec2, x);
            if constexpr (HW) wt = weights[k];
        };
        constexpr uint64_t B = kSegBlock;
        uint64_t i = begin + threadIdx.x;  // this thread's tuples: i, i + B, i + 2B, ...
        uint32_t xn[G][NC];
        int64_t wn[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            wn[g] = 0;
            if (i + g * B < end) load(i + g * B, xn[g], wn[g]);
        }
        for (; i + (G - 1) * B < end; i += G * B) {  // a whole group
            uint32_t x[G][NC];
            int64_t wt[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int c = 0; c < NC; ++c) x[g][c] = xn[g][c];
                wt[g] = wn[g];
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (i + (G + g) * B < end) load(i + (G + g) * B, xn[g], wn[g]);
            uint32_t j[G], neg[G], flag = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                uint32_t f;
                hash1(x[g], j[g], neg[g], f);
                flag = max(flag, f);
            }
            if (flag >= canon_thresh) {  // a hash may need the full reduction
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    uint32_t jj, nn, f;
                    hash1(x[g], jj, nn, f);
                    if (f >= canon_thresh) exact1(x[g], j[g], neg[g]);
                }
            }
            Pend now[G];
#pragma unroll
            for (int g = 0; g < G; ++g) now[g] = add1(j[g], neg[g], wt[g]);
            check();
#pragma unroll
            for (int g = 0; g < G; ++g) pend[g] = now[g];
        }
        // fewer than G tuples left, one at a time (their keys are in xn)
#pragma unroll
        for (int g = 0; g < G - 1; ++g) {
            if (i + g * B < end) {
                uint32_t jj, nn, f;
                hash1(xn[g], jj, nn, f);
                if (f >= canon_thresh) exact1(xn[g], jj, nn);
                const Pend now = add1(jj, nn, wn[g]);
                check();
                pend[0] = now;
#pragma unroll
                for (int h = 1; h < G; ++h) pend[h] = Pend{kBias16 * 0x10001u, 0u, 0u, s_w};
            }
        }
        check();
    }
    __syncthreads();
    // partial sums leave as the biased 16-bit pairs: [chunk][cells / 2] words
    uint32_t *out = partial + (size_t)wg.chunk * (cells >> 1) + (cell0 >> 1);
    for (uint32_t e = threadIdx.x; e < span / 2; e += kSegBlock) out[e] = s_w[e];
}

// The same 16-bit update for relations of one or two key columns when one repetition
// fills the segment (R = m): a thread takes quads of four consecutive tuples, so a quad's
// keys arrive in one 16-byte load per column pair (A16: keys and weights 16-byte aligned;
// otherwise one load per key).  The next quad's loads are issued before the current quad
// is hashed, at an index clamped into the chunk instead of behind a branch; the tuples
// after the chunk's last whole quad (at most three) go one per thread at the end.  The
// loop is unrolled twice so that the two quads' keys alternate between two register sets
// without copies.  A quad's four returned words are checked right after its adds (the
// other wavefronts of the SIMD cover the LDS latency; deferring the check to the next quad
// measured slower, its register copies outweighing the wait).
template <int NC, bool E1, bool HW, bool A16>
__global__ __launch_bounds__(kSegBlock) void k_update_seg16q(const uint32_t *__restrict__ keys,
                                                             const int64_t *__restrict__ weights, uint64_t n,
                                                             const uint64_t *__restrict__ coef, int32_t cpr,
                                                             DevPlan plan, uint32_t m, uint64_t chunk,
                                                             uint32_t *partial, unsigned long long *sketch,
                                                             uint32_t canon_thresh,
                                                             const unsigned long long *__restrict__ n_dev)
{
    if (n_dev) {  // tuple count known only on the device (a filtered update's kept tuples)
        n = *n_dev;
        chunk = ((n + gridDim.x - 1) / gridDim.x + 3) & ~(uint64_t)3;
    }
    static_assert(NC == 1 || NC == 2, "quads of one- and two-column tuples");
    __shared__ uint32_t s_w[kSeg16Words];
    const uint64_t cells = (uint64_t)gridDim.y * m;  // one segment per repetition
    const SegTile wg = seg_tile();
    const int t = (int)wg.seg;
    for (uint32_t e = threadIdx.x; e < m / 2; e += kSegBlock) s_w[e] = (kBias16 << 16) | kBias16;
    __syncthreads();
    const uint64_t begin = (uint64_t)wg.chunk * chunk;  // chunk is a multiple of 4
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    const uint64_t len = end > begin ? end - begin : 0;
    const uint64_t nq = len >> 2;
    const uint64_t *cf = coef + (size_t)t * cpr;
    CoefE1<NC> K;
    if constexpr (E1) K.load(cf);
    unsigned long long *srow = sketch + (uint64_t)t * m;

    struct Quad {
        uint32_t x[4][NC];
        int64_t w[4];
    };
    struct Pend {
        uint32_t old, inc, j;  // word before the add, the increment, the bucket
    };
    auto load_quad = [&](uint64_t q, Quad &Q) {
        const uint64_t i0 = begin + 4 * q;
        if constexpr (A16) {
            const uint4 *p = reinterpret_cast<const uint4 *>(keys + i0 * NC);
            if constexpr (NC == 1) {
                const uint4 v = p[0];
                Q.x[0][0] = v.x;
                Q.x[1][0] = v.y;
                Q.x[2][0] = v.z;
                Q.x[3][0] = v.w;
            } else {
                const uint4 a = p[0], b = p[1];
                Q.x[0][0] = a.x;
                Q.x[0][1] = a.y;
                Q.x[1][0] = a.z;
                Q.x[1][1] = a.w;
                Q.x[2][0] = b.x;
                Q.x[2][1] = b.y;
                Q.x[3][0] = b.z;
                Q.x[3][1] = b.w;
            }
            if constexpr (HW) {
                const longlong2 *pw = reinterpret_cast<const longlong2 *>(weights + i0);
                const longlong2 u = pw[0], v = pw[1];
                Q.w[0] = u.x;
                Q.w[1] = u.y;
                Q.w[2] = v.x;
                Q.w[3] = v.y;
            }
        } else {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
#pragma unroll
                for (int c = 0; c < NC; ++c) Q.x[g][c] = keys[(i0 + g) * NC + c];
                if constexpr (HW) Q.w[g] = weights[i0 + g];
            }
        }
        if constexpr (!HW) {
#pragma unroll
            for (int g = 0; g < 4; ++g) Q.w[g] = 1;
        }
    };
    auto hash1 = [&](const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg, uint32_t &flag) {
        if constexpr (E1) {
            K.bin_neg_fast(x, j, neg, flag);
        } else {
            hash_rep<NC>(cf, plan, x, j, neg);
            flag = 0;
        }
    };
    auto exact1 = [&](const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg) {
        if constexpr (E1) {
            j = K.bin(x);
            neg = K.neg(x);
        }
    };
    // j is the bucket before the mask (E1) or reduced (otherwise); the word's byte offset
    // masks and scales in two instructions, and the half's shift uses only bit 0 of j
    const uint32_t word_mask = E1 ? 2 * m - 4 : ~3u;
    auto add1 = [&](uint32_t j, uint32_t neg, int64_t wt) -> Pend {
        if constexpr (HW) neg ^= (uint32_t)((uint64_t)wt >> 63);
        uint32_t sgn;  // 1 - 2 neg in one instruction
        asm("v_mad_i32_i24 %0, %1, -2, 1" : "=v"(sgn) : "v"(neg));
        const uint32_t inc = sgn << ((j & 1u) << 4);  // inc16(neg, bit 0 of j)
        uint32_t *w = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(s_w) + ((j << 1) & word_mask));
        return Pend{atomicAdd(w, inc), inc, j};
    };
    // out16 of four adds at once: every word's both halves must show the window bit
    auto check = [&](const Pend (&P)[4]) {
        uint32_t all = 0x80008000u;
#pragma unroll
        for (int g = 0; g < 4; ++g) all &= P[g].old + P[g].inc + 0x40004000u;
        if (all != 0x80008000u) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
                if (out16(P[g].old, P[g].inc)) {
                    const uint32_t jm = E1 ? P[g].j & (m - 1) : P[g].j;
                    spill16(&s_w[jm >> 1], shift16(P[g].inc), srow + jm);
                }
        }
    };
    auto process = [&](const Quad &Q, Pend (&P)[4]) {
        uint32_t j[4], neg[4], flag = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint32_t f;
            hash1(Q.x[g], j[g], neg[g], f);
            flag = max(flag, f);
        }
        if (flag >= canon_thresh) {  // a hash may need the full reduction
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                uint32_t jj, nn, f;
                hash1(Q.x[g], jj, nn, f);
                if (f >= canon_thresh) exact1(Q.x[g], j[g], neg[g]);
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) P[g] = add1(j[g], neg[g], Q.w[g]);
    };

    Pend P[4];
    if (nq > 0) {
        const uint64_t last = nq - 1;
        uint64_t q = threadIdx.x;
        Quad A, B;
        load_quad(q < last ? q : last, A);
        while (q < nq) {
            load_quad(q + kSegBlock < last ? q + kSegBlock : last, B);
            process(A, P);
            check(P);
            q += kSegBlock;
            if (q >= nq) break;
            load_quad(q + kSegBlock < last ? q + kSegBlock : last, A);
            process(B, P);
            check(P);
            q += kSegBlock;
        }
    }
    // the chunk's last len mod 4 tuples, one per thread
    if ((uint64_t)threadIdx.x < (len & 3)) {
        const uint64_t i = begin + 4 * nq + threadIdx.x;
        uint32_t x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = keys[i * NC + c];
        const int64_t wt = HW ? weights[i] : 1;
        uint32_t j, neg, f;
        hash1(x, j, neg, f);
        if (f >= canon_thresh) exact1(x, j, neg);
        Pend one[4];
        one[0] = add1(j, neg, wt);
#pragma unroll
        for (int g = 1; g < 4; ++g) one[g] = Pend{kBias16 * 0x10001u, 0u, 0u};
        check(one);
    }
    __syncthreads();
    uint32_t *out = partial + (size_t)wg.chunk * (cells >> 1) + (((uint64_t)t * m) >> 1);
    for (uint32_t e = threadIdx.x; e < m / 2; e += kSegBlock) out[e] = s_w[e];
}

// 16-bit counters beyond 2^16 buckets (m a power of two, one or two key columns, each in
// one join, Deltas +-1): a workgroup owns a range of 2^16 buckets of one repetition.
// Each wavefront hashes the bins of 64 tuples (the fast reduction, exact when flagged),
// queues those whose bucket falls in the range (keys, offset in the range, sign of
// Delta) in LDS and hashes their signs only once 64 are queued, so the sign work runs
// at full SIMD width; every tuple's bin is hashed once per range of its repetition,
// its sign once.  Each add's returned word is checked right away (one unchecked add per
// thread).  Partial sums leave as biased 16-bit pairs, like k_update_seg16q's.
template <int NC, bool HW>
__global__ __launch_bounds__(kSegBlock) void k_update_seg16c(const uint32_t *__restrict__ keys,
                                                             const int64_t *__restrict__ weights, uint64_t n,
                                                             const uint64_t *__restrict__ coef, int32_t cpr,
                                                             uint32_t m, uint64_t chunk, bool vec2,
                                                             uint32_t *partial, unsigned long long *sketch,
                                                             uint32_t canon_thresh)
{
    static_assert(NC == 1 || NC == 2, "one- and two-column relations");
    constexpr uint32_t kRange = 1u << 16;
    constexpr int kWavesPB = kSegBlock / 64;
    __shared__ uint32_t s_w[kSeg16Words];
    __shared__ uint32_t s_qx[kWavesPB][NC][kQCap];
    __shared__ uint32_t s_ql[kWavesPB][kQCap];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t cells = (uint64_t)gridDim.y * kRange;  // d * m
    const SegTile wg = seg_tile();
    const uint64_t cell0 = (uint64_t)wg.seg * kRange;
    const int t = (int)(cell0 / m);
    const uint32_t off = (uint32_t)(cell0 - (uint64_t)t * m);  // first bucket of the range
    for (uint32_t e = threadIdx.x; e < kSeg16Words; e += kSegBlock) s_w[e] = (kBias16 << 16) | kBias16;
    __syncthreads();
    CoefE1<NC> K;
    K.load(coef + (size_t)t * cpr);
    unsigned long long *srow = sketch + (uint64_t)t * m + off;
    const uint64_t begin = (uint64_t)wg.chunk * chunk;
    const uint64_t end = begin + chunk < n ? begin + chunk : n;
    // bin and sign without the canonical reduction (CoefE1::bin_neg_fast split in two)
    auto bin_fast = [&](const uint32_t (&x)[NC], uint32_t &flag) {
        uint32_t j = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const HPair rb = hstep_p(hpair(K.b1[c]), x[c], K.b0[c]);
            j += rb.lo + (rb.hi >> 29);
            flag = max(flag, rb.hi | 0xE0000000u);
        }
        return j;
    };
    auto neg_fast = [&](const uint32_t (&x)[NC], uint32_t &flag) {
        uint32_t neg = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const HPair rs = hstep_p(hstep_p(hstep_p(hpair(K.a[c][3]), x[c], K.a[c][2]), x[c], K.a[c][1]), x[c],
                                     K.a[c][0]);
            neg ^= rs.lo ^ (rs.hi >> 29);
            flag = max(flag, rs.hi | 0xE0000000u);
        }
        return neg & 1u;
    };
    uint32_t head = 0, count = 0;  // wave-uniform queue state
    auto drain = [&](uint32_t k) {  // lanes < k take one queued tuple each
        if ((uint32_t)lane < k) {
            const uint32_t slot = (head + lane) & (kQCap - 1);
            uint32_t x[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = s_qx[wave][c][slot];
            const uint32_t l = s_ql[wave][slot];
            uint32_t flag = 0;
            uint32_t neg = neg_fast(x, flag);
            if (flag >= canon_thresh) neg = K.neg(x);
            neg ^= l >> 31;
            const uint32_t j = l & (kRange - 1);
            const uint32_t inc = inc16(neg, (j & 1u) << 4);
            uint32_t *w = &s_w[j >> 1];
            const uint32_t old = atomicAdd(w, inc);
            if (out16(old, inc)) spill16(w, shift16(inc), srow + j);
        }
        head = (head + k) & (kQCap - 1);
        count -= k;
    };
    for (uint64_t base = begin + (uint64_t)wave * 64; base < end; base += kSegBlock) {
        const uint64_t i = base + lane;
        bool in = false;
        uint32_t x[NC], loc = 0;
        if (i < end) {
            load_keys<NC>(keys, i, vec2, x);
            uint32_t flag = 0;
            uint32_t j = bin_fast(x, flag);
            if (flag >= canon_thresh) j = K.bin(x);
            j = (j & (m - 1)) - off;
            if (j < kRange) {
                in = true;
                loc = j | ((HW && weights[i] < 0) ? 0x80000000u : 0u);
            }
        }
        const uint64_t mask = __ballot(in);
        if (in) {
            const uint32_t pos = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            const uint32_t slot = (head + count + pos) & (kQCap - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) s_qx[wave][c][slot] = x[c];
            s_ql[wave][slot] = loc;
        }
        count += (uint32_t)__popcll(mask);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (count >= 64) drain(64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (count > 0) drain(count);
    __syncthreads();
    uint32_t *out = partial + (size_t)wg.chunk * (cells >> 1) + (cell0 >> 1);
    for (uint32_t e = threadIdx.x; e < kSeg16Words; e += kSegBlock) out[e] = s_w[e];
}

// Compaction pass of a filtered update with 16-bit counters: the keys (and Deltas) of the
// tuples that pass f are written contiguously to okeys / ow, and their number is added to
// *count (and to *kept when set).  A workgroup takes a tile of kPB x 16 tuples: each
// wavefront loads the attribute columns and keys of its 16 groups of 64 consecutive
// tuples at once, evaluates the predicates (one ballot per group), and the workgroup
// reserves its tile's slots with one atomic.  The kept tuples' order is not kept: the
// counters, integer sums, do not depend on it.  Each tuple's predicates are evaluated
// once here, instead of once per repetition in the update kernel.
constexpr int kCB = 256;  // compaction workgroup: 4 wavefronts
template <int NC, bool HW, int MAXP>
__global__ __launch_bounds__(kCB) void k_filter_compact(const uint32_t *__restrict__ keys,
                                                        const int64_t *__restrict__ weights, uint64_t n,
                                                        const uint32_t *__restrict__ attrs, int32_t n_attrs,
                                                        FilterSpec f, bool vec2, uint32_t *okeys, int64_t *ow,
                                                        unsigned long long *count, unsigned long long *kept)
{
    // groups of 64 tuples per wavefront and tile: all their loads are issued before the
    // first predicate is evaluated (at most MAXP attribute values held per tuple)
    constexpr int kG = MAXP > 2 ? 4 : 16;
    __shared__ uint32_t s_cnt[kCB / 64];
    __shared__ unsigned long long s_base[kCB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t tile = (uint64_t)kCB * kG;
    const int np = f.n;
    for (uint64_t t0 = (uint64_t)blockIdx.x * tile; t0 < n; t0 += (uint64_t)gridDim.x * tile) {
        const uint64_t g0 = t0 + (uint64_t)wave * 64 * kG;
        uint32_t av[kG][MAXP];
        uint32_t x[kG][NC];
        int64_t w[kG];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const uint64_t i = g0 + (uint64_t)g * 64 + lane;
            const uint64_t ic = i < n ? i : n - 1;  // clamped: every load stays in bounds
#pragma unroll
            for (int p = 0; p < MAXP; ++p)
                if (p < np) av[g][p] = attrs[ic * (uint64_t)n_attrs + f.col[p]];
            load_keys<NC>(keys, ic, vec2, x[g]);
            if constexpr (HW) w[g] = weights[ic];
        }
        uint64_t bal[kG];
        uint32_t total = 0;
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            bool in = g0 + (uint64_t)g * 64 + lane < n;
#pragma unroll
            for (int p = 0; p < MAXP; ++p)
                if (p < np) in = in && av[g][p] >= f.lo[p] && av[g][p] <= f.hi[p];
            bal[g] = __ballot(in);
            total += (uint32_t)__popcll(bal[g]);
        }
        if (lane == 0) s_cnt[wave] = total;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t sum = 0;
            for (int v = 0; v < kCB / 64; ++v) sum += s_cnt[v];
            unsigned long long b = sum ? atomicAdd(count, (unsigned long long)sum) : 0ull;
            if (kept && sum) atomicAdd(kept, (unsigned long long)sum);
            for (int v = 0; v < kCB / 64; ++v) {
                s_base[v] = b;
                b += s_cnt[v];
            }
        }
        __syncthreads();
        unsigned long long o = s_base[wave];
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            if ((bal[g] >> lane) & 1ull) {
                const uint64_t dst = o + (uint64_t)__popcll(bal[g] & ((1ull << lane) - 1ull));
                if constexpr (NC == 2) {
                    reinterpret_cast<uint2 *>(okeys)[dst] = make_uint2(x[g][0], x[g][1]);
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) okeys[dst * NC + c] = x[g][c];
                }
                if constexpr (HW) ow[dst] = w[g];
            }
            o += (uint64_t)__popcll(bal[g]);
        }
        __syncthreads();  // s_cnt / s_base are rewritten by the next tile
    }
}

// sketch[2w + h] += sum over chunks of (half h of partial[chunk][w]) - 2^15
// reset, when set, is a device count the update kernel has finished reading (a filtered
// update's kept tuples): it is set back to zero for the handle's next filtered update.
__global__ void k_seg_reduce16(const uint32_t *__restrict__ partial, int32_t C, uint64_t words,
                               unsigned long long *sketch, unsigned long long *reset = nullptr)
{
    if (reset && blockIdx.x == 0 && threadIdx.x == 0) *reset = 0ull;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words;
         w += (uint64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = 0;
#pragma unroll 8
        for (int c = 0; c < C; ++c) {
            const uint32_t v = partial[(size_t)c * words + w];
            lo += (int64_t)(v & 0xFFFFu);
            hi += (int64_t)(v >> 16);
        }
        lo -= (int64_t)C * kBias16;
        hi -= (int64_t)C * kBias16;
        sketch[2 * w] += (unsigned long long)lo;
        sketch[2 * w + 1] += (unsigned long long)hi;
    }
}

// sketch[cell] += sum over chunks of partial[chunk][cell] (int64, wrapping)
template <typename CT>
__global__ void k_seg_reduce(const CT *__restrict__ partial, int32_t C, uint64_t cells, uint64_t *sketch)
{
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cells;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t s = 0;
        for (int c = 0; c < C; ++c) s += (uint64_t)(int64_t)partial[(size_t)c * cells + e];
        sketch[e] += s;
    }
}

// ---------------------------------------------------------------- sort by bucket range
//
// Partition strategy for m beyond what one workgroup's LDS holds (and any m when asked
// for): every (tuple, repetition) is hashed exactly once into a 16-bit record, the
// records are grouped by (repetition, bucket range of 2^14 buckets), and one workgroup
// per group sums them in LDS and adds the sums into the int64 counters it alone owns.
// Deltas must be +1 (weights NULL) or +-1 (flag CS_UPDATE_UNIT_WEIGHTS).  The tuples
// run in chunks of at most kPartMaxChunk (two kernels per chunk).
//
// Pass 1 (k_part_hash): a workgroup owns a block of kPartBlk consecutive tuples; each
// of its four wavefronts loads the keys of its quarter once (quads of consecutive
// tuples per lane, 16-byte loads) and the workgroup loops over a group of repetitions.
// Per repetition every wavefront hashes its tuples and ranks them per bucket range in
// its own LDS histogram (the add's returned value is the record's rank; four
// sub-histograms by lane & 3 keep a wavefront's lanes apart); one scan across ranges
// and wavefronts places each range's run, padded to a multiple of four records, in the
// block's LDS staging area; the block's records and run starts leave coalesced.
//
// Zipf-skewed keys put a large share of a stream on a few tuples; left alone, pass 2's
// LDS adds on their buckets would serialise (same-address atomics) and the workgroup of
// their range would carry most records.  Each block therefore elects up to kPartHot hot
// tuples (sixteen candidates: the relation's hints, the hottest tuples of its previous
// update, then the first tuples of lanes of every wavefront; counted over the first four
// quads of the block's lanes and kept when they hold at least 8 of those 1024 tuples),
// sums their Deltas instead of emitting records for them, and leaves (tuple, Delta sum)
// in a list that pass 2 hashes once per repetition.  The sketch is linear (Sec. 2.2): n
// equal tuples with Deltas Delta_i add sum_i Delta_i at their one counter, so the
// counters are unchanged whichever tuples are elected.  Sixteen sampled tuples alone
// miss a key of 6% of the stream in a third of the blocks; the hints carry the stream's
// heavy keys from one update call to the next.
//
// Pass 2 (k_part_accum): workgroup (range r, repetition t) zeroes two copies of 2^14
// int32 LDS counters (even and odd lanes add to different copies, which halves the
// lanes of one add that meet on a skewed bucket's word), adds +-1 for every record of
// its group from every block (8-byte loads of four records, four runs in flight per
// wavefront), adds the hot tuples whose bucket falls in its range, and adds the non-zero
// sums of the two copies into the sketch (it owns those counters: plain
// read-modify-write, no atomics).  One extra workgroup writes the relation's hints: the
// distinct hot tuples of the first eight blocks, ranked by their |Delta sum| over all
// blocks.

constexpr int kPartLog2R = 14;                   // buckets per range (pass-2 LDS: two copies of 2^14 int32, 128 KB)
constexpr uint32_t kPartR = 1u << kPartLog2R;
constexpr int kPartQuads = 4;                    // quads of tuples per lane
constexpr int kPartSlots = 4 * kPartQuads;       // tuples per lane
constexpr int kPartWave = 64 * kPartSlots;       // 1024 tuples per wavefront
constexpr int kPB = 256;                         // pass-1 workgroup: 4 wavefronts
constexpr int kPartBlk = kPartWave * (kPB / 64); // 4096 tuples per block
constexpr int kPartBlkCap = kPartBlk + 4 * 64;   // records of a block and repetition, runs padded to 4
constexpr int kPartHS = 4;                       // sub-histograms per range
constexpr int kPAB = 1024;                       // pass-2 workgroup
constexpr uint32_t kPartNone = 0xFFFFFFFFu;      // an empty hot-table entry
constexpr uint32_t kPartHotMin = 8;              // sample hits (of 1024) for a hot tuple
// Word of a slot in pass 1: record (15 bits: offset in its range, sign) | 0 (bit 15) |
// range (bits 16-22) | rank in its sub-histogram (bits 23-30, < 256).  A slot without a
// record carries range kPartSinkRange, whose sub-histogram entries permanently point at
// the staging area's sink entries, so placement needs no test.
constexpr uint32_t kPartSinkRange = 64;
constexpr uint32_t kPartSink = kPartSinkRange << 16;
constexpr uint16_t kPartPad = 0xFFFFu;           // padding record (bit 15 set: never a real one)
static_assert(kMaxPartRanges <= 64, "one lane per bucket range");
static_assert(kPartBlkCap <= 0xFFFF && kPartBlkCap % 8 == 0, "16-bit run starts, 16-byte stores");
static_assert(sizeof(PartHot) == 12 * kPartHot, "hot-tuple entry layout");

template <int NC>
__device__ __forceinline__ bool same_key(const uint32_t (&a)[NC], const uint32_t (&b)[NC])
{
    bool e = true;
#pragma unroll
    for (int c = 0; c < NC; ++c) e = e && a[c] == b[c];
    return e;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wavefront: in-row steps by DPP row shifts
// of 1, 2, 4 and 8 lanes, then the row broadcasts of lane 15 (into rows 1 and 3) and of
// lane 31 (into rows 2 and 3); a lane without a source adds 0.  All lanes must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Entry of a tuple in the direct-mapped table of a block's hot tuples (multiplicative
// hashing of the key words).
constexpr int kPartHotTab = 256;
template <int NC>
__device__ __forceinline__ uint32_t part_hot_slot(const uint32_t (&x)[NC])
{
    uint32_t h = x[0] * 0x9E3779B1u;
    if constexpr (NC == 2) h ^= x[1] * 0x85EBCA77u;
    return h >> 24;  // 256 entries
}

// Bucket j in [0, m) and sign bit of one tuple for one repetition: the one-join fast
// hash (m a power of two; the full reduction only when a hash's flag asks for it, see
// CoefE1::bin_neg_fast), or the general one (any m, any joins per column).
template <int NC, bool FAST>
struct PartHasher {
    CoefE1<NC> K;
    const uint64_t *cf;
    DevPlan plan;
    uint32_t mmask;
    __device__ __forceinline__ void load(const uint64_t *coef_t)
    {
        cf = coef_t;
        if constexpr (FAST) K.load(coef_t);
    }
    __device__ __forceinline__ void hash(const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg, uint32_t &flag) const
    {
        if constexpr (FAST) {
            K.bin_neg_fast(x, j, neg, flag);
        } else {
            hash_rep<NC>(cf, plan, x, j, neg);
            flag = 0;
        }
    }
    __device__ __forceinline__ void exact(const uint32_t (&x)[NC], uint32_t &j, uint32_t &neg) const
    {
        if constexpr (FAST) {
            j = K.bin(x);
            neg = K.neg(x);
        }
    }
    __device__ __forceinline__ uint32_t bucket(uint32_t j) const { return FAST ? (j & mmask) : j; }
};

// Pass 1.  Grid (blocks, repetition groups), mapped by seg_tile() so that the groups of
// one block share an XCD (its L2 fetches the keys once).
template <int NC, bool FAST, bool HW, bool A16, bool FILT>
__global__ __launch_bounds__(kPB, 4) void k_part_hash(const uint32_t *__restrict__ keys,
                                                         const int64_t *__restrict__ weights, uint64_t n,
                                                         const uint64_t *__restrict__ coef, int32_t cpr,
                                                         DevPlan plan, uint32_t m, int32_t d, int32_t ranges,
                                                         int32_t reps_per_group, uint64_t nblk, uint16_t *rec_out,
                                                         uint16_t *tab, PartHot *hot, uint32_t canon_thresh,
                                                         const uint32_t *__restrict__ attrs, int32_t n_attrs,
                                                         FilterSpec f, unsigned long long *kept,
                                                         const PartHints *__restrict__ hints)
{
    static_assert(NC == 1 || NC == 2, "one- and two-column relations");
    __shared__ __align__(16) uint32_t s_hist[kPB / 64][(kPartSinkRange + 1) * kPartHS];
    __shared__ uint32_t s_tot[kPB / 64][64];
    __shared__ __align__(16) uint16_t s_stage[kPartBlkCap + 64];  // + one sink entry per lane
    const SegTile wg = seg_tile();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t blk = wg.chunk;
    const int t0 = (int)wg.seg * reps_per_group;
    const int t1 = min(d, t0 + reps_per_group);
    const uint64_t base = blk * kPartBlk + (uint64_t)wave * kPartWave;
    const bool full = base + kPartWave <= n;

    // ---- keys of this wavefront's quarter: slot s = 4 q + g is tuple base + 4 (64 q + lane) + g
    uint32_t x[kPartSlots][NC];
    uint32_t valid = 0, wneg = 0;  // bit s: slot s holds a tuple / its Delta is -1
#pragma unroll
    for (int q = 0; q < kPartQuads; ++q) {
        const uint64_t i0 = base + 4 * ((uint64_t)q * 64 + lane);
        if (A16 && full) {
            const uint4 *p = reinterpret_cast<const uint4 *>(keys + i0 * NC);
            if constexpr (NC == 1) {
                const uint4 v = p[0];
                x[4 * q + 0][0] = v.x;
                x[4 * q + 1][0] = v.y;
                x[4 * q + 2][0] = v.z;
                x[4 * q + 3][0] = v.w;
            } else {
                const uint4 a = p[0], b = p[1];
                x[4 * q + 0][0] = a.x;
                x[4 * q + 0][1] = a.y;
                x[4 * q + 1][0] = a.z;
                x[4 * q + 1][1] = a.w;
                x[4 * q + 2][0] = b.x;
                x[4 * q + 2][1] = b.y;
                x[4 * q + 3][0] = b.z;
                x[4 * q + 3][1] = b.w;
            }
            if constexpr (HW) {
                const longlong2 *pw = reinterpret_cast<const longlong2 *>(weights + i0);
                const longlong2 u = pw[0], v = pw[1];
                wneg |= ((uint32_t)((uint64_t)u.x >> 63) | ((uint32_t)((uint64_t)u.y >> 63) << 1) |
                         ((uint32_t)((uint64_t)v.x >> 63) << 2) | ((uint32_t)((uint64_t)v.y >> 63) << 3))
                        << (4 * q);
            }
            valid |= 0xFu << (4 * q);
        } else {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint64_t i = i0 + g;
                const bool in = i < n;
                const uint64_t ic = in ? i : 0;  // clamped: every load stays in bounds
#pragma unroll
                for (int c = 0; c < NC; ++c) x[4 * q + g][c] = keys[ic * NC + c];
                if constexpr (HW) wneg |= (uint32_t)((uint64_t)weights[ic] >> 63) << (4 * q + g);
                valid |= (uint32_t)in << (4 * q + g);
            }
        }
    }
    wneg &= valid;
    // With a filter, the kept tuples of this wavefront's quarter are compacted (through
    // LDS) into its first ceil(kept / 64) slots, and the repetition loop hashes only those.
    int nslots = kPartSlots;
    if constexpr (FILT) {
        extern __shared__ __align__(16) uint32_t s_list[];  // [waves][NC + HW][kPartWave]
        constexpr int kW = NC + (HW ? 1 : 0);
        uint32_t *lst = s_list + (size_t)wave * kW * kPartWave;
        uint32_t off = 0;
#pragma unroll
        for (int q = 0; q < kPartQuads; ++q) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int sl = 4 * q + g;
                const uint64_t i = base + 4 * ((uint64_t)q * 64 + lane) + g;
                const bool kp = ((valid >> sl) & 1u) && passes(attrs, n_attrs, i, f);
                const uint64_t bal = __ballot(kp);
                if (kp) {
                    const uint32_t dst = off + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
#pragma unroll
                    for (int c = 0; c < NC; ++c) lst[c * kPartWave + dst] = x[sl][c];
                    if constexpr (HW) lst[NC * kPartWave + dst] = (wneg >> sl) & 1u;
                }
                off += (uint32_t)__popcll(bal);
            }
        }
        wave_sync();
        const uint32_t total = off;
        nslots = (int)((total + 63) / 64);
        valid = 0;
        wneg = 0;
#pragma unroll
        for (int sl = 0; sl < kPartSlots; ++sl) {
            const uint32_t e = (uint32_t)sl * 64 + lane;
            const bool in = e < total;
#pragma unroll
            for (int c = 0; c < NC; ++c) x[sl][c] = in ? lst[c * kPartWave + e] : 0u;
            if constexpr (HW) wneg |= (in ? lst[NC * kPartWave + e] : 0u) << sl;
            valid |= (uint32_t)in << sl;
        }
        if (kept && wg.seg == 0 && lane == 0 && total) atomicAdd(kept, (unsigned long long)total);
    }

    // ---- hot tuples of the block (see above)
    constexpr int kCand = kPB / 64 * 4;
    __shared__ uint32_t s_cand[kCand][NC];
    __shared__ uint32_t s_ccnt[kPB / 64][kCand];
    __shared__ uint32_t s_hot[kPartHot][NC];
    __shared__ int32_t s_hsum[kPB / 64][kPartHot];
    __shared__ int32_t s_nh;
    __shared__ uint4 s_htab[kPartHotTab];  // key(s), index into s_hot (kPartNone: empty)
    // candidates: the relation's hints from its previous update, then sampled tuples
    // (the first of lanes 0-3 of every wavefront, lane-major, while room is left)
    const int nhint = hints ? (int)min(hints->n, (uint32_t)kPartHot) : 0;
    if (threadIdx.x < nhint) {
#pragma unroll
        for (int c = 0; c < NC; ++c) s_cand[threadIdx.x][c] = hints->key[threadIdx.x][c];
    }
    if (lane < 4 && nhint + lane * 4 + wave < kCand) {
#pragma unroll
        for (int c = 0; c < NC; ++c) s_cand[nhint + lane * 4 + wave][c] = x[0][c];
    }
    for (int e = threadIdx.x; e < kPartHotTab; e += kPB) s_htab[e] = make_uint4(0u, 0u, kPartNone, 0u);
    __syncthreads();
    for (int ci = 0; ci < kCand; ++ci) {
        uint32_t kc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) kc[c] = s_cand[ci][c];
        uint32_t cnt = 0;
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) cnt += (uint32_t)__popcll(__ballot(((valid >> sl) & 1u) && same_key<NC>(x[sl], kc)));
        if (lane == 0) s_ccnt[wave][ci] = cnt;
    }
    __syncthreads();
    if (wave == 0) {
        // candidates by total count over the 1024 sampled tuples, distinct keys, at
        // least kPartHotMin hits, the kPartHot hottest (ties: lower candidate index); lane
        // ci < kCand holds candidate ci.  A candidate enters the direct-mapped table
        // unless a hotter elected one has the same entry (it stays an ordinary tuple);
        // entries are numbered in hotness order.
        const int ci = lane < kCand ? lane : 0;
        uint32_t kc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) kc[c] = s_cand[ci][c];
        uint32_t v = 0;
        for (int w = 0; w < kPB / 64; ++w) v += s_ccnt[w][ci];
        for (int cj = 0; cj < ci; ++cj) {
            bool same = true;
#pragma unroll
            for (int c = 0; c < NC; ++c) same = same && s_cand[cj][c] == kc[c];
            v = same ? 0u : v;
        }
        if (lane >= kCand) v = 0;
        int rank = 0;
#pragma unroll
        for (int cj = 0; cj < kCand; ++cj) {
            const uint32_t vj = __shfl(v, cj, 64);
            rank += (vj > v || (vj == v && cj < ci)) ? 1 : 0;
        }
        const bool elig = lane < kCand && rank < kPartHot && v >= kPartHotMin;
        const uint32_t slot = part_hot_slot<NC>(kc);
        bool blocked = false;
        int idx = 0;
#pragma unroll
        for (int cj = 0; cj < kCand; ++cj) {
            const int rj = __shfl(rank, cj, 64);
            const bool ej = __shfl((int)elig, cj, 64) != 0;
            const uint32_t sj = __shfl(slot, cj, 64);
            blocked = blocked || (ej && rj < rank && sj == slot);
        }
        const bool ins = elig && !blocked;
        // entry number: the inserted candidates of lower rank
#pragma unroll
        for (int cj = 0; cj < kCand; ++cj) {
            const int rj = __shfl(rank, cj, 64);
            const bool ij = __shfl((int)ins, cj, 64) != 0;
            idx += (ij && rj < rank) ? 1 : 0;
        }
        if (ins) {
            s_htab[slot] = make_uint4(kc[0], kc[NC - 1], (uint32_t)idx, 0u);
#pragma unroll
            for (int c = 0; c < NC; ++c) s_hot[idx][c] = kc[c];
        }
        const uint64_t bal = __ballot(ins);
        if (lane == 0) s_nh = (int32_t)__popcll(bal);
    }
    __syncthreads();
    const int nh = s_nh;
    uint32_t live = valid;  // slots that emit records
    if (nh > 0) {
        // each tuple probes one entry of a direct-mapped LDS table of the hot tuples
        // (thread 0 placed them; a hot tuple whose entry was taken stays an ordinary
        // one) and hot ones add their Delta to their tuple's sum
        if (lane < kPartHot) s_hsum[wave][lane] = 0;
        wave_sync();
        for (int sl = 0; sl < kPartSlots; ++sl) {
            if (!((valid >> sl) & 1u)) continue;
            const uint4 e = s_htab[part_hot_slot<NC>(x[sl])];
            const bool mt = e.z != kPartNone && e.x == x[sl][0] && (NC == 1 || e.y == x[sl][NC - 1]);
            if (mt) {
                atomicAdd(&s_hsum[wave][e.z], ((wneg >> sl) & 1u) ? -1 : 1);
                live &= ~(1u << sl);
            }
        }
        // A wavefront whose hot tuples free at least one group of slots gathers its
        // other tuples into its first slots: their indices in its quarter (and Delta
        // signs) pass through the staging area, unused before the repetition loop, and
        // their keys are loaded again (from L2), so that the repetition loop hashes
        // ceil(live / 64) slots instead of all (a hot tuple's buckets are hashed once,
        // in pass 2).  One-column relations only: for two columns the extra registers
        // cost the unskewed case 2% and the skewed case gained about as much (pairs of
        // keys are far less concentrated than single keys).
        if constexpr (!FILT && NC == 1) {
            constexpr int G = NC == 1 ? 4 : 2;
            uint32_t tl = 0;
#pragma unroll
            for (int sl = 0; sl < kPartSlots; ++sl) tl += (uint32_t)__popcll(__ballot((live >> sl) & 1u));
            if (tl <= 64u * (kPartSlots - G)) {
                uint16_t *li = s_stage + wave * kPartWave;
                uint32_t off = 0;
#pragma unroll
                for (int sl = 0; sl < kPartSlots; ++sl) {
                    const bool lv = (live >> sl) & 1u;
                    const uint64_t bal = __ballot(lv);
                    if (lv) {
                        const uint32_t dst = off + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                        const uint32_t q = (uint32_t)sl >> 2, g = (uint32_t)sl & 3u;
                        li[dst] = (uint16_t)((4u * (64u * q + (uint32_t)lane) + g) | (((wneg >> sl) & 1u) << 15));
                    }
                    off += (uint32_t)__popcll(bal);
                }
                wave_sync();
                nslots = (int)((tl + 63u) / 64u);
                valid = 0;
                wneg = 0;
#pragma unroll
                for (int sl = 0; sl < kPartSlots; ++sl) {
                    const uint32_t e = (uint32_t)sl * 64u + (uint32_t)lane;
                    const bool in = e < tl;
                    const uint32_t w = in ? (uint32_t)li[e] : 0u;
                    const uint64_t i = base + (w & 0x7FFFu);  // a valid tuple of this quarter when in
#pragma unroll
                    for (int c = 0; c < NC; ++c) x[sl][c] = 0u;
                    if (sl < nslots && in) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) x[sl][c] = keys[i * NC + c];
                    }
                    wneg |= (w >> 15) << sl;
                    valid |= (uint32_t)in << sl;
                }
                live = valid;
            }
        }
    }
    __syncthreads();
    if (wg.seg == 0 && threadIdx.x < kPartHot) {
        const int k = threadIdx.x;
        int32_t v = 0;
        if (k < nh)
            for (int w = 0; w < kPB / 64; ++w) v += s_hsum[w][k];
        PartHot *h = hot + blk;
        h->key[k][0] = k < nh ? s_hot[k][0] : 0u;
        h->key[k][1] = k < nh ? s_hot[k][NC - 1] : 0u;
        h->sum[k] = v;
    }

    // ---- per repetition: hash, rank by range, scan, scatter, store
    PartHasher<NC, FAST> hs;
    hs.plan = plan;
    hs.mmask = m - 1;
    uint32_t *hist = s_hist[wave];
    const uint32_t sub = lane & (kPartHS - 1);
    // byte offset of this lane's sub-histogram column of range 0 within s_hist
    const uint32_t hsub = (uint32_t)(((uintptr_t)(hist + sub)) - (uintptr_t)&s_hist[0][0]);
    if (lane < kPartHS) hist[kPartSinkRange * kPartHS + lane] = (uint32_t)kPartBlkCap + lane;  // never cleared
    // a bucket b = j & (m - 1) (one-join hash) or j: range b >> 14 as one bit-field
    // extract of j, position within the range j & min(m - 1, 2^14 - 1)
    const uint32_t log2m = 31u - (uint32_t)__builtin_clz(m);  // m a power of two when FAST
    const uint32_t rbits = FAST ? (log2m > kPartLog2R ? log2m - kPartLog2R : 0u) : 32u - kPartLog2R;
    const uint32_t pmask = FAST ? min(m - 1, kPartR - 1) : kPartR - 1;
    for (int t = t0; t < t1; ++t) {
        hs.load(coef + (size_t)t * cpr);
        reinterpret_cast<uint4 *>(hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
        wave_sync();
        uint32_t P[kPartSlots];
        // tuples hashed together: four one-column or two two-column tuples (eight or
        // four independent Horner chains) keep the register count within 128
        constexpr int G = NC == 1 ? 4 : 2;
#pragma unroll
        for (int q = 0; q < kPartSlots / G; ++q) {
            if ((FILT || NC == 1) && G * q >= nslots) {  // no kept or live tuple in these slots (wave-uniform)
#pragma unroll
                for (int g = 0; g < G; ++g) P[G * q + g] = kPartSink;
                continue;
            }
            uint32_t j[G], ng[G], flag = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                uint32_t f;
                hs.hash(x[G * q + g], j[g], ng[g], f);
                flag = max(flag, f);
            }
            if (flag >= canon_thresh) {  // a hash may need the full reduction
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    uint32_t jj, nn, f;
                    hs.hash(x[G * q + g], jj, nn, f);
                    if (f >= canon_thresh) hs.exact(x[G * q + g], j[g], ng[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int s = G * q + g;
                P[s] = kPartSink;
                if ((live >> s) & 1u) {
                    const uint32_t r = __builtin_amdgcn_ubfe(j[g], kPartLog2R, rbits);
                    const uint32_t rc = (j[g] & pmask) | (((ng[g] ^ (wneg >> s)) & 1u) << kPartLog2R);
                    // the counts are kept times 2^23, so the rank (< 256) comes back in place
                    const uint32_t pos23 = atomicAdd(&hist[r * kPartHS + sub], 1u << 23);
                    P[s] = rc | (r << 16) | pos23;
                }
            }
        }
        wave_sync();
        // run of range L: this wavefront's four sub-counts, their prefix, the totals of
        // every wavefront; the block's runs padded to multiples of four records
        const uint4 h4 = reinterpret_cast<const uint4 *>(hist)[lane];
        const uint32_t e1 = h4.x >> 23, e2 = e1 + (h4.y >> 23), e3 = e2 + (h4.z >> 23), tot = e3 + (h4.w >> 23);
        s_tot[wave][lane] = tot;
        __syncthreads();
        uint32_t before = 0, rtot = 0;
#pragma unroll
        for (int w = 0; w < kPB / 64; ++w) {
            const uint32_t v = s_tot[w][lane];
            before += w < wave ? v : 0u;
            rtot += v;
        }
        const uint32_t padded = (rtot + 3u) & ~3u;
        const uint32_t incl = wave_incl_scan(padded);
        const uint32_t start = incl - padded;
        const uint32_t wb = start + before;
        reinterpret_cast<uint4 *>(hist)[lane] = make_uint4(wb, wb + e1, wb + e2, wb + e3);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (wave == 0) {
            uint16_t *tb = tab + ((uint64_t)t * nblk + blk) * (uint64_t)(ranges + 1);
            if (lane < ranges) tb[lane] = (uint16_t)start;
            if (lane == 0) tb[ranges] = (uint16_t)total;
            for (uint32_t e = start + rtot; e < start + padded; ++e) s_stage[e] = kPartPad;
        }
        wave_sync();
        // placement, eight slots at a time: their run bases are read before any of
        // their records is written (a slot without a record reads its sub-histogram's
        // sink entry and writes a sink entry of the staging area, never stored)
#pragma unroll
        for (int s0 = 0; s0 < kPartSlots; s0 += 8) {
            uint32_t at[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                // LDS byte address of the slot's sub-histogram entry: range * 16 + hsub in
                // two instructions
                uint32_t a;
                asm("v_bfe_u32 %0, %1, 16, 7\n\tv_lshl_add_u32 %0, %0, 4, %2" : "=&v"(a) : "v"(P[s0 + s]), "v"(hsub));
                at[s] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(s_hist) + a);
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                // byte offset (at + rank) * 2 in one add-and-shift (bit 31 of a slot word is 0)
                uint32_t off;
                asm("v_add_lshl_u32 %0, %1, %2, 1" : "=v"(off) : "v"(at[s]), "v"(P[s0 + s] >> 23));
                *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(s_stage) + off) = (uint16_t)P[s0 + s];
            }
        }
        __syncthreads();
        uint4 *dst = reinterpret_cast<uint4 *>(rec_out + ((uint64_t)t * nblk + blk) * kPartBlkCap);
        const uint4 *src = reinterpret_cast<const uint4 *>(s_stage);
        for (uint32_t v = threadIdx.x; v * 8 < total; v += kPB) dst[v] = src[v];
        __syncthreads();
    }
}

// The relation's hints for its next update: candidates are the distinct hot tuples of
// the first eight blocks, each credited with the |Delta sum| of every block entry equal
// to it; the kPartHot largest non-zero totals, largest first (ties: lower candidate).
__device__ void part_hints(const PartHot *__restrict__ hot, uint64_t nblk, PartHints *out)
{
    constexpr int kHC = 8 * kPartHot;
    __shared__ uint32_t h_key[kHC][2];
    __shared__ uint32_t h_tot[kHC];
    __shared__ uint32_t h_ok[kHC];
    const int nc = (int)(nblk < 8 ? nblk : 8) * kPartHot;
    const int tid = threadIdx.x;
    if (tid < kHC) {
        uint32_t k0 = 0, k1 = 0, ok = 0;
        if (tid < nc) {
            const PartHot &h = hot[tid / kPartHot];
            k0 = h.key[tid % kPartHot][0];
            k1 = h.key[tid % kPartHot][1];
            ok = h.sum[tid % kPartHot] != 0 ? 1u : 0u;
        }
        h_key[tid][0] = k0;
        h_key[tid][1] = k1;
        h_ok[tid] = ok;
        h_tot[tid] = 0;
    }
    __syncthreads();
    bool live = false;
    if (tid < kHC) {
        live = h_ok[tid] != 0;
        for (int c = 0; c < tid && live; ++c)
            live = !(h_ok[c] && h_key[c][0] == h_key[tid][0] && h_key[c][1] == h_key[tid][1]);
    }
    __syncthreads();
    if (tid < kHC) h_ok[tid] = live ? 1u : 0u;
    __syncthreads();
    for (uint64_t e = tid; e < nblk * kPartHot; e += blockDim.x) {
        const PartHot &h = hot[e / kPartHot];
        const int k = (int)(e % kPartHot);
        const int32_t sm = h.sum[k];
        if (sm == 0) continue;
        const uint32_t k0 = h.key[k][0], k1 = h.key[k][1];
        for (int c = 0; c < nc; ++c)
            if (h_ok[c] && h_key[c][0] == k0 && h_key[c][1] == k1) {
                atomicAdd(&h_tot[c], (uint32_t)(sm < 0 ? -sm : sm));
                break;
            }
    }
    __syncthreads();
    if (tid < 64) {  // one wavefront ranks the kHC = 64 candidates
        const uint32_t v = h_ok[tid] ? h_tot[tid] : 0u;
        int rank = 0;
        for (int c = 0; c < kHC; ++c) {
            const uint32_t vc = __shfl(v, c, 64);
            rank += (vc > v || (vc == v && c < tid)) ? 1 : 0;
        }
        const bool take = v > 0 && rank < kPartHot;
        if (take) {
            out->key[rank][0] = h_key[tid][0];
            out->key[rank][1] = h_key[tid][1];
        }
        const uint64_t bal = __ballot(take);
        if (tid == 0) out->n = (uint32_t)__popcll(bal);
    }
}
static_assert(8 * kPartHot == 64, "one wavefront ranks the hint candidates");

// Pass 2.  Block (range r, repetition t).
template <int NC, bool FAST>
__global__ __launch_bounds__(kPAB) void k_part_accum(const uint16_t *__restrict__ rec,
                                                     const uint16_t *__restrict__ tab,
                                                     const PartHot *__restrict__ hot, uint64_t nblk,
                                                     int32_t ranges, uint32_t m, const uint64_t *__restrict__ coef,
                                                     int32_t cpr, DevPlan plan, uint64_t *sketch,
                                                     uint32_t canon_thresh, int32_t d, PartHints *hints_out)
{
    extern __shared__ __align__(16) uint32_t s_dyn[];
    if ((int)blockIdx.y == d) {  // the hints workgroup (row d of the grid: column 0 only)
        if (blockIdx.x == 0 && hints_out) part_hints(hot, nblk, hints_out);
        return;
    }
    // two copies of the counters, taken by even and odd lanes: the lanes of one add that
    // hit a skewed bucket's word are split over two words
    int32_t *s_cnt = reinterpret_cast<int32_t *>(s_dyn);   // [2][kPartR]
    uint32_t *s_run = s_dyn + 2 * kPartR;                   // [nblk]: start / 4 | words << 16
    const int r = blockIdx.x, t = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t *my_cnt = s_cnt + (lane & 1) * kPartR;
    constexpr int kWaves = kPAB / 64;
    constexpr int kInFlight = 4;  // runs per wavefront whose loads are issued together
    for (uint32_t e = threadIdx.x; e < 2 * kPartR / 4; e += kPAB) reinterpret_cast<int4 *>(s_cnt)[e] = make_int4(0, 0, 0, 0);
    for (uint64_t b = threadIdx.x; b < nblk; b += kPAB) {
        const uint16_t *tb = tab + ((uint64_t)t * nblk + b) * (uint64_t)(ranges + 1);
        const uint32_t beg = tb[r], end = tb[r + 1];  // multiples of 4
        s_run[b] = (beg >> 2) | (((end - beg) >> 2) << 16);
    }
    __syncthreads();
    auto add4 = [&](uint2 w) {
        const uint32_t v[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (v[k] != kPartPad) atomicAdd(&my_cnt[v[k] & (kPartR - 1)], (v[k] >> kPartLog2R) & 1u ? -1 : 1);
    };
    // records: wavefront w takes blocks w, w + kWaves, ..., kInFlight of them at a time;
    // a run of L words is read by lanes 0..L-1 (one 8-byte word of four records each)
    const uint2 *rt = reinterpret_cast<const uint2 *>(rec + (uint64_t)t * nblk * kPartBlkCap);
    for (uint64_t b0 = wave; b0 < nblk; b0 += (uint64_t)kWaves * kInFlight) {
        uint32_t run[kInFlight];
        const uint2 *p[kInFlight];
        uint32_t lmax = 0;
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const uint64_t b = b0 + (uint64_t)u * kWaves;
            run[u] = b < nblk ? s_run[b] : 0u;
            p[u] = rt + (b < nblk ? b : 0) * (kPartBlkCap / 4) + (run[u] & 0xFFFFu);
            lmax = max(lmax, run[u] >> 16);
        }
        for (uint32_t i = lane; i < lmax; i += 64) {
            uint2 w[kInFlight];
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) w[u] = i < (run[u] >> 16) ? p[u][i] : make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) add4(w[u]);
        }
    }
    // hot tuples of every wavefront quarter whose bucket falls in this range
    PartHasher<NC, FAST> hs;
    hs.plan = plan;
    hs.mmask = m - 1;
    hs.load(coef + (size_t)t * cpr);
    for (uint64_t e = threadIdx.x; e < nblk * kPartHot; e += kPAB) {
        const PartHot &h = hot[e / kPartHot];
        const int k = (int)(e % kPartHot);
        {
            if (h.sum[k] == 0) continue;
            uint32_t x[NC];
            x[0] = h.key[k][0];
            if constexpr (NC == 2) x[1] = h.key[k][1];
            uint32_t j, ng, f;
            hs.hash(x, j, ng, f);
            if (f >= canon_thresh) hs.exact(x, j, ng);
            const uint32_t b = hs.bucket(j);
            if ((int)(b >> kPartLog2R) == r) atomicAdd(&my_cnt[b & (kPartR - 1)], ng ? -h.sum[k] : h.sum[k]);
        }
    }
    __syncthreads();
    uint64_t *out = sketch + (uint64_t)t * m + ((uint64_t)r << kPartLog2R);
    const uint32_t span = min(kPartR, m - ((uint32_t)r << kPartLog2R));  // the last range may be partial
    for (uint32_t e = threadIdx.x; e < span; e += kPAB) {
        const int64_t v = (int64_t)s_cnt[e] + (int64_t)s_cnt[kPartR + e];
        if (v) out[e] += (uint64_t)v;
    }
}

}  // namespace
int32_t chunks_for_n(int32_t C, uint64_t n);
namespace {

template <int NC>
cs_status launch_nc(const UpdateArgs &a, int strategy, int grid_blocks, hipStream_t s)
{
    DevPlan plan{};
    for (int c = 0; c < kMaxCols; ++c) plan.n_edges[c] = c < a.plan.n_cols ? a.plan.n_edges[c] : 0;
    plan.bm = make_binmod(a.m);
    const bool pow2 = plan.bm.pow2 != 0;
    const bool vec2 = NC == 2 && ((uintptr_t)a.keys % 8) == 0;
    auto *sk = reinterpret_cast<unsigned long long *>(a.sketch);
    int dev = 0;
    CSK_HIP(hipGetDevice(&dev));
    int n_cu = 256;
    CSK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t need = (a.n + kBlock - 1) / kBlock;
    if (a.filter) {
        // Filtered ingestion: 16-bit LDS counters for m <= 2^16, the partition strategy
        // beyond (one-join columns, m a power of two, Deltas +-1, at most two columns);
        // global atomics for every other shape.
        bool e1 = pow2;
        for (int c = 0; c < a.plan.n_cols; ++c) e1 = e1 && a.plan.n_edges[c] == 1;
        const bool unit = a.weights == nullptr || a.unit_weights;
        if constexpr (NC <= 2) {
            if (e1 && unit && a.scratch && a.m > (1u << 16)) {
                strategy = CS_UPDATE_PARTITION;  // handled below with the filter
            } else if (e1 && unit && a.scratch && a.m > (1u << 15) && a.m % 2 == 0) {
                // one compaction pass per round (predicates evaluated once per tuple, kept
                // keys written contiguously, their count left on the device), then the
                // 16-bit quad kernel over the kept tuples, reading that count
                const uint64_t cells = (uint64_t)a.d * a.m;
                SegGeom g16 = seg16_geometry(a.m, a.d, a.scratch_bytes / 2, a.n);  // at most half for partial sums
                const size_t part_bytes = (((size_t)g16.chunks * cells * 2) + 255) & ~(size_t)255;
                const size_t per_tuple = (size_t)NC * 4 + (a.weights ? 8 : 0);
                if (part_bytes + 512 + 64 * per_tuple > a.scratch_bytes)
                    return fail(CS_EINVAL, "update scratch buffer too small for a filtered update");
                const uint64_t round_max = ((a.scratch_bytes - part_bytes - 512) / per_tuple) & ~(uint64_t)63;
                uint32_t *part = reinterpret_cast<uint32_t *>(a.scratch);
                // the handle's kept-tuple counter: zero between filtered updates (set at
                // creation, and back to zero by the reduction of every round)
                unsigned long long *cnt = a.filter_count;
                if (!cnt) return fail(CS_EINVAL, "filtered update without a device counter");
                uint32_t *okeys = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(a.scratch) + part_bytes + 256);
                const size_t wo = (((size_t)round_max * NC * 4) + 255) & ~(size_t)255;
                int64_t *ow = a.weights ? reinterpret_cast<int64_t *>(reinterpret_cast<char *>(okeys) + wo) : nullptr;
                if (a.weights && (part_bytes + 256 + wo + round_max * 8) > a.scratch_bytes)
                    return fail(CS_EINVAL, "update scratch buffer too small for a filtered update");
                const bool few = a.filter->n <= 2;
                auto ck = a.weights ? (few ? &k_filter_compact<NC, true, 2> : &k_filter_compact<NC, true, CS_MAX_PREDICATES>)
                                    : (few ? &k_filter_compact<NC, false, 2> : &k_filter_compact<NC, false, CS_MAX_PREDICATES>);
                const uint64_t tile = (uint64_t)kCB * (few ? 16 : 4);
                auto kern = a.weights ? &k_update_seg16q<NC, true, true, true> : &k_update_seg16q<NC, true, false, true>;
                dim3 grid16((unsigned)g16.chunks, (unsigned)g16.segments);
                if (g16.R != a.m || g16.segments != a.d) return fail(CS_EINVAL, "16-bit segment geometry");
                CSK_MARK(a.ev_start, s);
                for (uint64_t r0 = 0; r0 < a.n; r0 += round_max) {
                    const uint64_t rn = std::min<uint64_t>(a.n - r0, round_max);
                    const uint32_t *kb = a.keys + r0 * NC;
                    const bool v2 = NC == 2 && ((uintptr_t)kb % 8) == 0;
                    hipLaunchKernelGGL(ck, dim3((unsigned)std::min<uint64_t>((rn + tile - 1) / tile, 8192)), dim3(kCB), 0,
                                       s, kb, a.weights ? a.weights + r0 : nullptr, rn,
                                       a.attrs + r0 * (uint64_t)a.n_attrs, a.n_attrs, *a.filter, v2, okeys, ow, cnt,
                                       a.kept);
                    CSK_HIP(hipGetLastError());
                    hipLaunchKernelGGL(kern, grid16, dim3(kSegBlock), 0, s, okeys, ow, rn, a.coef, a.plan.coef_per_rep,
                                       plan, a.m, (uint64_t)4, part, sk, a.canon_thresh,
                                       (const unsigned long long *)cnt);
                    CSK_HIP(hipGetLastError());
                    const uint64_t words = cells / 2;
                    hipLaunchKernelGGL(k_seg_reduce16, dim3((unsigned)std::min<uint64_t>((words + 255) / 256, 8192)),
                                       dim3(256), 0, s, part, g16.chunks, words, sk, cnt);
                    CSK_HIP(hipGetLastError());
                }
                CSK_MARK(a.ev_stop, s);
                return CS_OK;
            }
        }
        if (strategy != CS_UPDATE_PARTITION) {
            uint64_t blocks = (uint64_t)n_cu * 16;
            if (blocks > need) blocks = need;
            CSK_MARK(a.ev_start, s);
            hipLaunchKernelGGL(k_update_global_f<NC>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a.keys, a.weights,
                               a.n, a.coef, a.plan.coef_per_rep, sk, a.m, a.d, plan, vec2, a.attrs, a.n_attrs,
                               *a.filter, a.kept);
            CSK_HIP(hipGetLastError());
            CSK_MARK(a.ev_stop, s);
            return CS_OK;
        }
    }
    if (strategy == CS_UPDATE_GLOBAL_ATOMIC || strategy == CS_UPDATE_WAVE_AGGREGATE) {
        uint64_t blocks = grid_blocks > 0 ? (uint64_t)grid_blocks : (uint64_t)n_cu * 16;
        if (blocks > need) blocks = need;
        CSK_MARK(a.ev_start, s);
        if (strategy == CS_UPDATE_GLOBAL_ATOMIC)
            hipLaunchKernelGGL(k_update_global<NC>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a.keys,
                               a.weights, a.n, a.coef, a.plan.coef_per_rep, sk, a.m, a.d, plan, vec2);
        else
            hipLaunchKernelGGL(k_update_waveagg<NC>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a.keys,
                               a.weights, a.n, a.coef, a.plan.coef_per_rep, sk, a.m, a.d, plan, vec2);
        CSK_HIP(hipGetLastError());
        CSK_MARK(a.ev_stop, s);
        return CS_OK;
    }
    if (strategy == CS_UPDATE_LDS_PRIVATE) {
        if (!a.scratch) return fail(CS_EINVAL, "LDS-segmented update needs a scratch buffer");
        // every Delta = +-1 and fewer than 2^31 tuples: int32 partial counters cannot overflow
        const bool narrow = (a.weights == nullptr || a.unit_weights) && a.n < (1ull << 31);
        const uint64_t cells = (uint64_t)a.d * a.m;
        // grid_blocks > 0 fixes the number of tuple chunks (bounded by the scratch buffer)
        auto chunks_for = [&](int32_t c, size_t elem) -> int32_t {
            if (grid_blocks <= 0) return c;
            const uint64_t cap = std::max<uint64_t>(1, a.scratch_bytes / (cells * elem));
            return (int32_t)std::min<uint64_t>((uint64_t)grid_blocks, std::min<uint64_t>(cap, 4096));
        };
        SegGeom sg = seg_geometry(a.m, a.d, narrow, a.scratch_bytes, a.n);
        sg.chunks = chunks_for(sg.chunks, narrow ? 4 : 8);
        const uint64_t chunk = (a.n + sg.chunks - 1) / sg.chunks;
        // every kernel below writes whole partial-sum planes: refuse a buffer they overrun
        auto fits = [&](int32_t chunks, size_t elem) { return (uint64_t)chunks * cells * elem <= a.scratch_bytes; };
        dim3 grid((unsigned)sg.chunks, (unsigned)sg.segments);
        const size_t lds = (size_t)sg.R * (narrow ? 4 : 8);
        int log2m = 0;
        while ((1u << log2m) < a.m) ++log2m;
        bool e1 = true;
        for (int c = 0; c < a.plan.n_cols; ++c) e1 = e1 && a.plan.n_edges[c] == 1;
        e1 = e1 && pow2;  // the one-join kernels reduce buckets by masking
        auto launch = [&](auto kern, auto *part) -> cs_status {
            CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            CSK_MARK(a.ev_start, s);
            hipLaunchKernelGGL(kern, grid, dim3(kSegBlock), lds, s, a.keys, a.weights, a.n, a.coef,
                               a.plan.coef_per_rep, plan, a.m, log2m, a.d, sg.R, chunk, vec2, part);
            CSK_HIP(hipGetLastError());
            CSK_MARK(a.ev_stop, s);
            return CS_OK;
        };
        cs_status st;
        if (narrow && a.m <= (1u << 16) && a.m > (1u << 15) && (a.m % 2) == 0 && a.counters16) {
            // 16-bit LDS counters: a whole repetition per workgroup
            SegGeom g16 = seg16_geometry(a.m, a.d, a.scratch_bytes, a.n);
            g16.chunks = chunks_for(g16.chunks, 2);
            if (!fits(g16.chunks, 2)) return fail(CS_EINVAL, "update scratch buffer too small for d * m 16-bit partial sums");
            dim3 grid16((unsigned)g16.chunks, (unsigned)g16.segments);
            if (g16.R > 2u * kSeg16Words) return fail(CS_EINVAL, "16-bit segment exceeds its LDS array");
            uint32_t *part = reinterpret_cast<uint32_t *>(a.scratch);
            auto *sk64 = reinterpret_cast<unsigned long long *>(a.sketch);
            CSK_MARK(a.ev_start, s);
            if constexpr (NC <= 2) {
                // quads of consecutive tuples: one repetition per segment, chunks of whole quads
                if (g16.R != a.m || g16.segments != a.d) return fail(CS_EINVAL, "16-bit segment geometry");
                const uint64_t chunkq = ((a.n + g16.chunks - 1) / g16.chunks + 3) & ~(uint64_t)3;
                const bool a16 = (reinterpret_cast<uintptr_t>(a.keys) & 15) == 0 &&
                                 (reinterpret_cast<uintptr_t>(a.weights) & 15) == 0;
                auto pick = [&](auto hw, auto al) {
                    constexpr bool HWv = decltype(hw)::value, ALv = decltype(al)::value;
                    return e1 ? &k_update_seg16q<NC, true, HWv, ALv> : &k_update_seg16q<NC, false, HWv, ALv>;
                };
                using T_ = std::true_type;
                using F_ = std::false_type;
                auto kern = a.weights ? (a16 ? pick(T_{}, T_{}) : pick(T_{}, F_{}))
                                      : (a16 ? pick(F_{}, T_{}) : pick(F_{}, F_{}));
                hipLaunchKernelGGL(kern, grid16, dim3(kSegBlock), 0, s, a.keys, a.weights, a.n, a.coef,
                                   a.plan.coef_per_rep, plan, a.m, chunkq, part, sk64, a.canon_thresh,
                                   (const unsigned long long *)nullptr);
            } else {
                const uint64_t chunk16 = (a.n + g16.chunks - 1) / g16.chunks;
                auto kern = a.weights ? (e1 ? &k_update_seg16<NC, true, true> : &k_update_seg16<NC, false, true>)
                                      : (e1 ? &k_update_seg16<NC, true, false> : &k_update_seg16<NC, false, false>);
                hipLaunchKernelGGL(kern, grid16, dim3(kSegBlock), 0, s, a.keys, a.weights, a.n, a.coef,
                                   a.plan.coef_per_rep, plan, a.m, log2m, a.d, g16.R, chunk16, vec2, part, sk64,
                                   a.canon_thresh);
            }
            CSK_HIP(hipGetLastError());
            CSK_MARK(a.ev_stop, s);
            const uint64_t words = cells / 2;
            hipLaunchKernelGGL(k_seg_reduce16, dim3((unsigned)std::min<uint64_t>((words + 255) / 256, 8192)),
                               dim3(256), 0, s, part, g16.chunks, words,
                               reinterpret_cast<unsigned long long *>(a.sketch), (unsigned long long *)nullptr);
        } else if (narrow && e1 && a.m > (1u << 16) && NC <= 2 && a.compact && a.counters16) {
            // 16-bit bucket ranges of 2^16 with compaction (e1 implies m a power of two)
            if constexpr (NC <= 2) {
                SegGeom gc = seg16_geometry(a.m, a.d, a.scratch_bytes, a.n);
                gc.chunks = chunks_for(gc.chunks, 2);
                if (!fits(gc.chunks, 2))
                    return fail(CS_EINVAL, "update scratch buffer too small for d * m 16-bit partial sums");
                if (gc.R != (1u << 16) || (uint64_t)gc.segments * gc.R != cells)
                    return fail(CS_EINVAL, "16-bit range geometry");
                const uint64_t chunkc = (a.n + gc.chunks - 1) / gc.chunks;
                uint32_t *part = reinterpret_cast<uint32_t *>(a.scratch);
                auto *sk64 = reinterpret_cast<unsigned long long *>(a.sketch);
                auto kern = a.weights ? &k_update_seg16c<NC, true> : &k_update_seg16c<NC, false>;
                CSK_MARK(a.ev_start, s);
                hipLaunchKernelGGL(kern, dim3((unsigned)gc.chunks, (unsigned)gc.segments), dim3(kSegBlock), 0, s,
                                   a.keys, a.weights, a.n, a.coef, a.plan.coef_per_rep, a.m, chunkc, vec2, part, sk64,
                                   a.canon_thresh);
                CSK_HIP(hipGetLastError());
                CSK_MARK(a.ev_stop, s);
                const uint64_t words = cells / 2;
                hipLaunchKernelGGL(k_seg_reduce16, dim3((unsigned)std::min<uint64_t>((words + 255) / 256, 8192)),
                                   dim3(256), 0, s, part, gc.chunks, words, sk64, (unsigned long long *)nullptr);
            }
        } else if (narrow && e1 && sg.R < a.m && NC <= 2 && a.compact) {
            // bucket-range segments: compacting kernel (queue after the counters in LDS)
            if (!fits(sg.chunks, 4)) return fail(CS_EINVAL, "update scratch buffer too small for d * m int32 partial sums");
            int32_t *part = reinterpret_cast<int32_t *>(a.scratch);
            const size_t lds_c = (size_t)sg.R * 4 + (size_t)(kSegBlock / 64) * (NC + 1) * kQCap * 4;
            CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_update_seg_compact<NC>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_c));
            CSK_MARK(a.ev_start, s);
            hipLaunchKernelGGL(k_update_seg_compact<NC>, grid, dim3(kSegBlock), lds_c, s, a.keys, a.weights, a.n,
                               a.coef, a.plan.coef_per_rep, a.m, log2m, a.d, sg.R, chunk, vec2, part);
            CSK_HIP(hipGetLastError());
            CSK_MARK(a.ev_stop, s);
            hipLaunchKernelGGL(k_seg_reduce<int32_t>, dim3((unsigned)std::min<uint64_t>((cells + 255) / 256, 8192)),
                               dim3(256), 0, s, reinterpret_cast<const int32_t *>(a.scratch), sg.chunks, cells,
                               a.sketch);
        } else if (narrow) {
            if (!fits(sg.chunks, 4)) return fail(CS_EINVAL, "update scratch buffer too small for d * m int32 partial sums");
            int32_t *part = reinterpret_cast<int32_t *>(a.scratch);
            st = e1 ? launch(&k_update_seg<NC, int32_t, true>, part) : launch(&k_update_seg<NC, int32_t, false>, part);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_seg_reduce<int32_t>, dim3((unsigned)std::min<uint64_t>((cells + 255) / 256, 8192)),
                               dim3(256), 0, s, reinterpret_cast<const int32_t *>(a.scratch), sg.chunks, cells,
                               a.sketch);
        } else {
            if (!fits(sg.chunks, 8)) return fail(CS_EINVAL, "update scratch buffer too small for d * m int64 partial sums");
            int64_t *part = reinterpret_cast<int64_t *>(a.scratch);
            st = e1 ? launch(&k_update_seg<NC, int64_t, true>, part) : launch(&k_update_seg<NC, int64_t, false>, part);
            if (st != CS_OK) return st;
            hipLaunchKernelGGL(k_seg_reduce<int64_t>, dim3((unsigned)std::min<uint64_t>((cells + 255) / 256, 8192)),
                               dim3(256), 0, s, reinterpret_cast<const int64_t *>(a.scratch), sg.chunks, cells,
                               a.sketch);
        }
        CSK_HIP(hipGetLastError());
        return CS_OK;
    }
    if (strategy == CS_UPDATE_PARTITION) {
        if constexpr (NC > 2) return fail(CS_EINVAL, "the partition strategy handles at most 2 key columns");
        else {
            if (a.weights && !a.unit_weights)
                return fail(CS_EINVAL, "the partition strategy needs weights NULL or flagged as +-1");
            if (!a.scratch) return fail(CS_EINVAL, "the partition strategy needs a scratch buffer");
            const PartGeom pg = part_geometry(a.m, a.d, a.scratch_bytes);
            if (pg.chunk == 0) return fail(CS_EINVAL, "scratch buffer too small for the partition strategy");
            bool fast = pow2;  // one-join columns and m a power of two: the fast hash
            for (int c = 0; c < a.plan.n_cols; ++c) fast = fast && a.plan.n_edges[c] == 1;
            uint16_t *rec = reinterpret_cast<uint16_t *>(a.scratch);
            uint16_t *tab = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(a.scratch) + pg.tab_offset);
            PartHot *hot = reinterpret_cast<PartHot *>(reinterpret_cast<char *>(a.scratch) + pg.hot_offset);
            // timing events: around the hashing pass when the call is one chunk, else
            // around both passes of every chunk
            const bool one_chunk = a.n <= pg.chunk;
            CSK_MARK(a.ev_start, s);
            for (uint64_t base = 0; base < a.n; base += pg.chunk) {
                const uint64_t cn = a.n - base < pg.chunk ? a.n - base : pg.chunk;
                const uint64_t nblk = (cn + kPartBlk - 1) / kPartBlk;
                const uint32_t *kb = a.keys + base * NC;
                const int64_t *wb = a.weights ? a.weights + base : nullptr;
                const bool a16 = (reinterpret_cast<uintptr_t>(kb) & 15) == 0 && (reinterpret_cast<uintptr_t>(wb) & 15) == 0;
                // repetition groups: within one round (at most four resident workgroups
                // per CU at 128 VGPRs), preferring at least three per CU to hide latency,
                // the split with the fewest repetitions per SIMD (workgroups per CU x
                // repetitions per workgroup); measured at 2^20 tuples, d = 15: three of
                // five repetitions beat four of four, four, four and three by 4%
                int groups = 1, per = a.d;
                {
                    uint64_t best = ~0ull;
                    for (int g = 1; g <= a.d; ++g) {
                        const int pg_ = (a.d + g - 1) / g, gg = (a.d + pg_ - 1) / pg_;
                        if (gg != g) continue;
                        const uint64_t k = (nblk * (uint64_t)gg + n_cu - 1) / n_cu;
                        if (g > 1 && k > 4) break;
                        // ties: fewer workgroups once three share a CU, else more
                        const uint64_t key = ((k >= 3 ? 0ull : 1ull) << 62) | ((k * (uint64_t)pg_) << 8) |
                                             (k >= 3 ? k : 255 - k);
                        if (key < best) {
                            best = key;
                            groups = gg;
                            per = pg_;
                        }
                    }
                }
                using T_ = std::true_type;
                using F_ = std::false_type;
                const bool filt = a.filter != nullptr;
                auto pick = [&](auto fst, auto hw, auto al) {
                    constexpr bool F = decltype(fst)::value, H = decltype(hw)::value, A = decltype(al)::value;
                    return filt ? &k_part_hash<NC, F, H, A, true> : &k_part_hash<NC, F, H, A, false>;
                };
                auto hk = fast ? (wb ? (a16 ? pick(T_{}, T_{}, T_{}) : pick(T_{}, T_{}, F_{}))
                                     : (a16 ? pick(T_{}, F_{}, T_{}) : pick(T_{}, F_{}, F_{})))
                               : (wb ? (a16 ? pick(F_{}, T_{}, T_{}) : pick(F_{}, T_{}, F_{}))
                                     : (a16 ? pick(F_{}, F_{}, T_{}) : pick(F_{}, F_{}, F_{})));
                // the filtered variant compacts each wavefront's kept tuples in LDS
                const size_t lds_f = filt ? (size_t)(kPB / 64) * (NC + (wb ? 1 : 0)) * kPartWave * 4 : 0;
                if (filt)
                    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(hk),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f));
                const uint32_t *ab = filt ? a.attrs + base * (uint64_t)a.n_attrs : nullptr;
                const FilterSpec fs = filt ? *a.filter : FilterSpec{};
                hipLaunchKernelGGL(hk, dim3((unsigned)nblk, (unsigned)groups), dim3(kPB), lds_f, s, kb, wb, cn, a.coef,
                                   a.plan.coef_per_rep, plan, a.m, a.d, pg.ranges, per, nblk, rec, tab, hot,
                                   a.canon_thresh, ab, a.n_attrs, fs, a.kept, a.hints);
                CSK_HIP(hipGetLastError());
                if (one_chunk) CSK_MARK(a.ev_stop, s);
                auto ak = fast ? &k_part_accum<NC, true> : &k_part_accum<NC, false>;
                const size_t lds = (size_t)kPartR * 8 + (size_t)nblk * 4;
                CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(ak),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                // grid row d: the workgroup that writes the relation's hints
                hipLaunchKernelGGL(ak, dim3((unsigned)pg.ranges, (unsigned)a.d + (a.hints ? 1u : 0u)), dim3(kPAB), lds,
                                   s, rec, tab, hot, nblk, pg.ranges, a.m, a.coef, a.plan.coef_per_rep, plan,
                                   a.sketch, a.canon_thresh, a.d, a.hints);
                CSK_HIP(hipGetLastError());
            }
            if (!one_chunk) CSK_MARK(a.ev_stop, s);
            return CS_OK;
        }
    }
    return fail(CS_EINVAL, "unknown update strategy");
}

}  // namespace

// At least this many tuples per chunk: a small update runs on fewer workgroups rather
// than paying each one's counter initialisation and partial-sum traffic.
constexpr uint64_t kSegTuplesPerChunk = 32768;

int32_t chunks_for_n(int32_t C, uint64_t n)
{
    const uint64_t by_n = n / kSegTuplesPerChunk + (n % kSegTuplesPerChunk != 0);  // no wrap at n = 2^64 - 1
    return (int32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)C, by_n));
}

SegGeom seg_geometry(uint32_t m, int32_t d, bool narrow, size_t scratch_bytes, uint64_t n)
{
    SegGeom g{};
    // LDS per block: 128 KB of counters (one 1024-thread block per CU)
    g.R = narrow ? (1u << 15) : (1u << 14);
    const uint64_t cells = (uint64_t)d * m;
    if (m <= g.R) g.R = (g.R / m) * m;  // whole repetitions per segment
    g.segments = (int32_t)((cells + g.R - 1) / g.R);
    // one 128 KB workgroup per CU: a whole number of rounds over the 256 CUs (two
    // rounds when there are few segments), bounded by the scratch buffer
    int32_t C = 512 / g.segments;
    if (C < 1) C = 1;
    const uint64_t cap = std::max<uint64_t>(1, scratch_bytes / (cells * (narrow ? 4 : 8)));
    if ((uint64_t)C > cap) C = (int32_t)cap;
    if (C > 64) C = 64;
    g.chunks = chunks_for_n(C, n);
    return g;
}

SegGeom seg16_geometry(uint32_t m, int32_t d, size_t scratch_bytes, uint64_t n)
{
    SegGeom g{};
    g.R = 1u << 16;  // 16-bit counters in 128 KB of LDS
    const uint64_t cells = (uint64_t)d * m;
    if (m <= g.R) g.R = (g.R / m) * m;
    g.segments = (int32_t)((cells + g.R - 1) / g.R);
    // one round of 128 KB workgroups over the 256 CUs: fewer partial sums to reduce
    int32_t C = 256 / g.segments;
    if (C < 1) C = 1;
    const uint64_t cap = std::max<uint64_t>(1, scratch_bytes / (cells * 2));
    if ((uint64_t)C > cap) C = (int32_t)cap;
    if (C > 64) C = 64;
    g.chunks = chunks_for_n(C, n);
    return g;
}

// Records (2 bytes per tuple and repetition, runs padded), run starts (2 bytes per range
// and repetition, plus a total) and the hot-tuple entries, per 4096-tuple block.
static size_t part_bytes_per_block(int32_t d, int32_t ranges)
{
    return (size_t)d * kPartBlkCap * 2 + (size_t)d * (ranges + 1) * 2 + sizeof(PartHot);
}

PartGeom part_geometry(uint32_t m, int32_t d, size_t scratch_bytes)
{
    PartGeom g{};
    g.ranges = (int32_t)(((uint64_t)m + kPartR - 1) >> kPartLog2R);
    if (g.ranges > kMaxPartRanges) return g;  // chunk 0: not applicable
    const size_t slack = 512;                 // two 256-byte alignments
    uint64_t nblk = scratch_bytes > slack ? (scratch_bytes - slack) / part_bytes_per_block(d, g.ranges) : 0;
    nblk = std::min<uint64_t>(nblk, kPartMaxChunk / kPartBlk);
    g.nseg = nblk;
    g.chunk = nblk * kPartBlk;
    // 256-byte aligned pieces: records, then run starts, then hot tuples
    const size_t rec_bytes = (size_t)d * nblk * kPartBlkCap * 2;
    const size_t tab_bytes = (size_t)d * nblk * (g.ranges + 1) * 2;
    g.tab_offset = (rec_bytes + 255) & ~(size_t)255;
    g.hot_offset = (g.tab_offset + tab_bytes + 255) & ~(size_t)255;
    return g;
}

size_t seg_scratch_bytes(uint32_t m, int32_t d)
{
    const uint64_t cells = (uint64_t)d * m;
    size_t best = 0;
    for (int narrow = 0; narrow < 2; ++narrow) {
        SegGeom g = seg_geometry(m, d, narrow != 0, (size_t)-1);
        best = std::max<size_t>(best, (size_t)g.chunks * cells * (narrow ? 4 : 8));
    }
    {
        const SegGeom g16 = seg16_geometry(m, d, (size_t)-1);
        best = std::max<size_t>(best, (size_t)g16.chunks * cells * 2);
    }
    // the partition strategy's chunk of kPartMaxChunk tuples where it is the automatic
    // choice (m > 2^16); below, chunks of 16 blocks (it runs there only when asked for)
    {
        const int32_t ranges = (int32_t)(((uint64_t)m + kPartR - 1) >> kPartLog2R);
        const uint64_t nblk = m > (1u << 16) ? kPartMaxChunk / kPartBlk : 16;
        best = std::max<size_t>(best, (size_t)nblk * part_bytes_per_block(d, ranges) + 512);
    }
    return best;
}

size_t update_scratch_bytes(uint32_t m, int32_t d, uint64_t n, bool unit)
{
    const uint64_t cells = (uint64_t)d * m;
    const bool narrow = unit && n < (1ull << 31);
    const SegGeom g = seg_geometry(m, d, narrow, (size_t)-1, n);
    size_t best = (size_t)g.chunks * cells * (narrow ? 4 : 8);
    if (unit) {
        const SegGeom g16 = seg16_geometry(m, d, (size_t)-1, n);
        best = std::max<size_t>(best, (size_t)g16.chunks * cells * 2);
        // partition: the blocks of one chunk of this input (up to kPartMaxChunk tuples
        // where it is the automatic choice, 16 blocks below 2^16 buckets)
        const int32_t ranges = (int32_t)(((uint64_t)m + kPartR - 1) >> kPartLog2R);
        const uint64_t cap = m > (1u << 16) ? kPartMaxChunk / kPartBlk : 16;
        const uint64_t nblk = std::min<uint64_t>(cap, n / kPartBlk + (n % kPartBlk != 0));
        best = std::max<size_t>(best, (size_t)nblk * part_bytes_per_block(d, ranges) + 512);
    }
    return best;
}

size_t filter_scratch_bytes(uint32_t m, int32_t d)
{
    // a filtered update with 16-bit counters (2^15 < m <= 2^16): the partial sums, then
    // the kept tuples' keys (and Deltas) in rounds of 2^23 tuples of two columns with
    // weights (16 bytes each), or 2^24 of two columns without
    if (m <= (1u << 15) || m > (1u << 16)) return 0;
    const SegGeom g16 = seg16_geometry(m, d, (size_t)-1);
    const size_t part = (size_t)g16.chunks * (size_t)d * m * 2;
    return std::max<size_t>(2 * part, part + ((size_t)16 << 23)) + 1024;
}

int auto_update_strategy(uint32_t m, int32_t d, uint64_t n, int n_cols, bool unit, bool has_scratch, bool e1_pow2)
{
    // Global atomics run at about 2.4e10/s on the whole chip (and far slower on the hot
    // buckets of skewed keys), the hash at about 5e12 Horner steps/s: beyond a few
    // microseconds of atomics the update aggregates in LDS, on as many chunks as the
    // input fills (seg_geometry).  Beyond 2^16 buckets a repetition no longer fits one
    // workgroup's LDS and each tuple's bucket would be hashed once per bucket range;
    // there the partition strategy (each tuple hashed once, records sorted by range)
    // measured 1.5-20x faster for m from 1.5 * 2^16 to 2^20, d from 3 to 9, than the int32
    // segments.  The 16-bit compacting kernel (ranges of 2^16 buckets, one-join columns,
    // m a power of two) beats it at two ranges per repetition (3e7 Zipf tuples, d = 5:
    // 0.82 vs 1.22 ms at m = 2^17) and loses from four on (m = 2^18, d = 5: 1.37 vs
    // 1.21 ms; d = 15: 4.5 vs 2.2 ms; 2^20: 5.7 vs 1.4 ms).  With general weights (no
    // partition) the int64 segments lose to wavefront-aggregated atomics beyond 2^18
    // buckets.
    if (!has_scratch) return CS_UPDATE_GLOBAL_ATOMIC;
    if (n * (uint64_t)d < 65536) return CS_UPDATE_GLOBAL_ATOMIC;
    if (m > (1u << 16) && unit && n_cols <= 2)
        return m <= (1u << 17) && d <= 9 && e1_pow2 ? CS_UPDATE_LDS_PRIVATE : CS_UPDATE_PARTITION;
    if (m > (1u << 18) && !unit) return CS_UPDATE_WAVE_AGGREGATE;
    return CS_UPDATE_LDS_PRIVATE;
}

namespace {

// One scratch buffer per device for callers without a buffer of their own (per-attribute
// sketches, the autotuner).  Reuse is stream-ordered while consecutive users share a
// stream; a user on another stream first drains the device.
struct ScratchPool {
    std::mutex mu;
    void *buf = nullptr;
    size_t bytes = 0;
    hipStream_t last_stream = nullptr;  // stream of the last user
    bool used = false;
};
std::mutex g_pool_mu;
std::map<int, ScratchPool *> g_pools;

ScratchPool &pool_of(int device)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    ScratchPool *&p = g_pools[device];
    if (!p) p = new ScratchPool();
    return *p;
}

cs_status dispatch_nc(const UpdateArgs &a, int strategy, int grid_blocks, hipStream_t s)
{
    switch (a.plan.n_cols) {
        case 1: return launch_nc<1>(a, strategy, grid_blocks, s);
        case 2: return launch_nc<2>(a, strategy, grid_blocks, s);
        case 3: return launch_nc<3>(a, strategy, grid_blocks, s);
        case 4: return launch_nc<4>(a, strategy, grid_blocks, s);
        case 5: return launch_nc<5>(a, strategy, grid_blocks, s);
        case 6: return launch_nc<6>(a, strategy, grid_blocks, s);
        case 7: return launch_nc<7>(a, strategy, grid_blocks, s);
        case 8: return launch_nc<8>(a, strategy, grid_blocks, s);
        default: return fail(CS_EINVAL, "relation has an unsupported number of key columns");
    }
}

}  // namespace

cs_status launch_update(const UpdateArgs &a_in, int strategy, int grid_blocks, hipStream_t s)
{
    if (a_in.n == 0) return CS_OK;
    UpdateArgs a = a_in;
    const bool unit = a.weights == nullptr || a.unit_weights;
    int dev = 0;
    CSK_HIP(hipGetDevice(&dev));
    if (strategy == CS_UPDATE_AUTO) {
        int ts = 0, tg = 0, tf = 0;
        if (tune_lookup(a, dev, &ts, &tg, &tf)) {  // the autotuner's choice for this class
            strategy = ts;
            grid_blocks = tg;
            a.compact = a.compact && (tf & CS_UPDATE_NO_COMPACT) == 0;
            a.counters16 = a.counters16 && (tf & CS_UPDATE_NO_COUNTERS16) == 0;
        } else {
            bool e1_pow2 = (a.m & (a.m - 1)) == 0;
            for (int c = 0; c < a.plan.n_cols; ++c) e1_pow2 = e1_pow2 && a.plan.n_edges[c] == 1;
            strategy = auto_update_strategy(a.m, a.d, a.n, a.plan.n_cols, unit, true, e1_pow2);
        }
    }
    if (strategy != CS_UPDATE_LDS_PRIVATE && strategy != CS_UPDATE_PARTITION) return dispatch_nc(a, strategy, grid_blocks, s);
    // A caller-owned scratch buffer (a handle's, allocated with it; or the static one of
    // the allocation-free entry point): its uses are ordered like the caller's updates.
    if (a.scratch) return dispatch_nc(a, strategy, grid_blocks, s);
    ScratchPool &P = pool_of(dev);
    std::lock_guard<std::mutex> lk(P.mu);
    const size_t need = seg_scratch_bytes(a.m, a.d);
    if (P.bytes < need) {
        // grows to the largest (m, d) seen by callers without a buffer of their own
        CSK_HIP(hipDeviceSynchronize());
        if (P.buf) (void)hipFree(P.buf);
        P.buf = nullptr;
        P.bytes = 0;
        if (hipMalloc(&P.buf, need) != hipSuccess) return fail(CS_ENOMEM, "update scratch allocation failed");
        P.bytes = need;
        P.used = false;
    }
    // Consecutive users on one stream are ordered by it: no event or marker per call.
    // On a change of stream the device is drained first (the previous stream may since
    // have been destroyed, so nothing is recorded on it).
    if (P.used && s != P.last_stream) CSK_HIP(hipDeviceSynchronize());
    a.scratch = P.buf;
    a.scratch_bytes = P.bytes;
    const cs_status st = dispatch_nc(a, strategy, grid_blocks, s);
    P.used = true;
    P.last_stream = s;
    return st;
}

}  // namespace csk

namespace csk {
namespace {
__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }
}  // namespace

cs_status zero_device_u64(unsigned long long *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}
}  // namespace csk

// ---------------------------------------------------------------- allocation-free update
//
// For callers that cannot allocate device memory while they run (code under graph
// capture, tight serving loops): the update's scratch buffer is this file-scope device
// array instead of the handle's.  Every GPU the library runs on holds one copy, at its
// own address, until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is taken once per device with
// hipGetSymbolAddress and only that address is ever handed to kernels.

constexpr size_t kStaticScratchBytes = 64ull << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace csk {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
cs_status static_scratch(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(CS_EINVAL, "device id beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_static_ptr[device] = p;
    }
    *out = g_static_ptr[device];
    return CS_OK;
}

}  // namespace
}  // namespace csk

extern "C" {

size_t cs_update_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

cs_status cs_update_noalloc(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                            int32_t flags, void *stream)
{
    using namespace csk;
    UpdateArgs a;
    cs_status st = update_args(hs, rel, keys, weights, n, flags & CS_UPDATE_UNIT_WEIGHTS, &a);
    if (st != CS_OK || n == 0) return st;
    int dev = -1;
    CSK_HIP(hipGetDevice(&dev));
    if (dev != hs->h.device) return fail(CS_EINVAL, "the handle's device must be the current device");
    void *p = nullptr;
    st = static_scratch(dev, &p);
    if (st != CS_OK) return st;
    a.scratch = p;
    a.scratch_bytes = kStaticScratchBytes;
    // the kernels fully write every partial sum and record they later read, so nothing
    // left in the array by an earlier call is ever read; a geometry the array cannot hold
    // is refused inside the launcher (CS_EINVAL) before anything is enqueued
    return launch_update(a, CS_UPDATE_AUTO, 0, static_cast<hipStream_t>(stream));
}

}  // extern "C"
