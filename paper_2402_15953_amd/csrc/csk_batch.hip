// Batched mode: thousands of uneven queries' updates in one persistent launch, and
// their estimates in one batched pass (estimate_batch).
//
// The update work list is cut into tasks: a tuple range of one relation of one query,
// and, for relations with many tuples per counter, one LDS segment of its [d][m]
// counters.  A persistent grid (one 1024-thread workgroup per CU, 128 KB LDS) pulls
// tasks from an atomic counter, largest first:
//   segment task - LDS counters of the segment (int32 when every Delta is +-1), the
//                  range's tuples hashed (bins first; signs only for in-segment buckets
//                  when the segment is a bucket range), then the non-zero counters are
//                  added into the sketch with one global atomic each;
//   atomic task  - few tuples per counter: one global atomic per tuple and repetition;
//   sort-reduce task - each wavefront takes 64 tuples at a time and, per repetition,
//                  sorts their 64 (counter, value) pairs across its lanes, sums the runs
//                  of equal counters and adds each run with one global atomic (skewed
//                  keys then meet in registers instead of on a counter's cache line).
// Counters are int64 and all adds commute, so the result is bit-identical to the plain
// per-query path whatever the task kind or order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <map>
#include <tuple>
#include <cstring>
#include <new>
#include <vector>

#include "csk_counters16.h"
#include "csk_handle.h"
#include "csk_hash.h"
#include "csk_internal.h"

namespace csk {

namespace {

constexpr int kBBlock = 1024;
constexpr size_t kBLds = 128 * 1024;

struct BItem {
    const uint32_t *keys;
    const int64_t *weights;
    const uint64_t *coef;
    uint64_t *sketch;
    uint64_t n;
    int32_t cpr;
    int32_t n_cols;
    uint32_t m;
    int32_t log2m;
    int32_t d;
    uint32_t R;        // cells per segment (segment tasks)
    int32_t narrow;    // int32 LDS counters (Deltas +-1)
    int32_t vec2;      // two-column keys 8-byte aligned
    int32_t e1;        // every key column in exactly one join and m a power of two
    DevPlan plan;
};

struct BTask {
    int32_t item;
    int32_t kind;      // 0: atomic, 1: LDS segment, 2: sort-reduce
    uint32_t seg;
    uint32_t pad;
    uint64_t begin, end;
};

__global__ void k_zero_u32(unsigned int *p) { *p = 0u; }

template <int NC>
__device__ void run_atomic(const BItem &I, uint64_t begin, uint64_t end)
{
    for (uint64_t i = begin + threadIdx.x; i < end; i += kBBlock) {
        uint32_t x[NC];
        load_keys<NC>(I.keys, i, I.vec2 != 0, x);
        const int64_t delta = I.weights ? I.weights[i] : 1;
        const uint64_t *cf = I.coef;
        for (int t = 0; t < I.d; ++t, cf += I.cpr) {
            uint32_t j, neg;
            hash_rep<NC>(cf, I.plan, x, j, neg);
            const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
            atomicAdd(reinterpret_cast<unsigned long long *>(I.sketch) + (size_t)t * I.m + j,
                      (unsigned long long)val);
        }
    }
}

// Sort-reduce task.  The loop over 64-tuple groups is uniform in each wavefront, so every
// lane takes part in every exchange; lanes past the range carry an empty counter index
// that sorts last and is never added.  Bitonic network over the 64 lanes: in stage
// (k, jj) lane l exchanges with l ^ jj and keeps the smaller index when it is the lower
// lane of an ascending pair (l & k == 0) or the upper lane of a descending one.  Equal
// indices are never exchanged, so both lanes of a pair always decide alike.  The sums are
// taken mod 2^64, as every counter add is.
template <int NC>
__device__ void run_sortreduce(const BItem &I, uint64_t begin, uint64_t end)
{
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // above every bucket (m <= 2^20)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long *sk = reinterpret_cast<unsigned long long *>(I.sketch);
    for (uint64_t g0 = begin + (uint64_t)wave * 64; g0 < end; g0 += (uint64_t)kBBlock) {
        const uint64_t i = g0 + lane;
        const bool valid = i < end;
        uint32_t x[NC];
        if (valid) {
            load_keys<NC>(I.keys, i, I.vec2 != 0, x);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = 0u;
        }
        const int64_t delta = valid ? (I.weights ? I.weights[i] : 1) : 0;
        const uint64_t *cf = I.coef;
        for (int t = 0; t < I.d; ++t, cf += I.cpr) {
            uint32_t j, neg;
            hash_rep<NC>(cf, I.plan, x, j, neg);
            uint32_t key = valid ? j : kEmpty;
            uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
#pragma unroll
            for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    const uint32_t ok = __shfl_xor(key, jj, 64);
                    const uint64_t ov = __shfl_xor(val, jj, 64);
                    const bool asc = (lane & k) == 0;
                    const bool low = (lane & jj) == 0;
                    if (low == asc ? ok < key : ok > key) {
                        key = ok;
                        val = ov;
                    }
                }
            }
            // inclusive sums within runs of equal indices (a run is contiguous once sorted)
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t uk = __shfl_up(key, o, 64);
                const uint64_t uv = __shfl_up(val, o, 64);
                if (lane >= o && uk == key) val += uv;
            }
            const uint32_t nk = __shfl_down(key, 1, 64);
            if ((lane == 63 || nk != key) && key != kEmpty && val != 0)
                atomicAdd(sk + (size_t)t * I.m + key, (unsigned long long)val);
        }
    }
}

template <int NC, typename CT>
__device__ void run_segment(const BItem &I, uint32_t seg, uint64_t begin, uint64_t end, CT *s_c)
{
    const uint64_t cells = (uint64_t)I.d * I.m;
    const uint64_t cell0 = (uint64_t)seg * I.R;
    const uint64_t cell1 = cell0 + I.R < cells ? cell0 + I.R : cells;
    const uint32_t span = (uint32_t)(cell1 - cell0);
    const int t0 = (int)(cell0 / I.m);
    const int t1 = (int)((cell1 - 1) / I.m);
    const bool whole = I.R >= I.m;
    for (uint32_t e = threadIdx.x; e < span; e += kBBlock) s_c[e] = 0;
    __syncthreads();
    for (uint64_t i = begin + threadIdx.x; i < end; i += kBBlock) {
        uint32_t x[NC];
        load_keys<NC>(I.keys, i, I.vec2 != 0, x);
        const int64_t delta = I.weights ? I.weights[i] : 1;
        for (int t = t0; t <= t1; ++t) {
            const uint64_t *cf = I.coef + (size_t)t * I.cpr;
            uint32_t j, neg;
            if (whole) {
                hash_rep<NC>(cf, I.plan, x, j, neg);
            } else {
                j = hash_bin<NC>(cf, I.plan, x);
                const uint64_t flat = (uint64_t)t * I.m + j;
                if (flat < cell0 || flat >= cell1) continue;
                neg = hash_neg<NC>(cf, I.plan, x);
            }
            const uint32_t loc = (uint32_t)(((uint64_t)t * I.m + j) - cell0);
            if constexpr (sizeof(CT) == 4) {
                const int32_t v32 = (int32_t)delta;
                atomicAdd(&s_c[loc], neg ? -v32 : v32);
            } else {
                const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
                atomicAdd(reinterpret_cast<unsigned long long *>(&s_c[loc]), (unsigned long long)val);
            }
        }
    }
    __syncthreads();
    unsigned long long *out = reinterpret_cast<unsigned long long *>(I.sketch) + cell0;
    for (uint32_t e = threadIdx.x; e < span; e += kBBlock) {
        const int64_t v = (int64_t)s_c[e];
        if (v) atomicAdd(out + e, (unsigned long long)v);
    }
    __syncthreads();
}

// Segment task with exact 16-bit counters (every Delta +-1): R = 2^16 counters in
// 128 KB, whole repetitions when m <= 2^16.  Keys of the next tuple are loaded while
// this one is hashed, and each LDS add's returned value is checked one add later.
// At the end, each non-zero counter is added into the sketch with one global atomic.
// Whole repetitions in the segment, one or two key columns: a thread takes quads of four
// consecutive tuples (loaded at an index clamped into the range, so no bounds branches),
// and per repetition hashes the quad in one straight-line block, issues its four LDS adds
// and checks the returned words right away (the other wavefronts cover the LDS latency).
// E1 (every column in exactly one join, m a power of two): coefficients in registers and
// the canonical reduction skipped unless a hash's flag asks for it.  The range's last
// (end - begin) mod 4 tuples go one per thread.
// Values the whole workgroup shares, moved into scalar registers (the compiler cannot
// tell that fields read from the task table are uniform).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v)
{
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
template <typename T>
__device__ __forceinline__ T *uni(T *p)
{
    return reinterpret_cast<T *>(uni(reinterpret_cast<uint64_t>(p)));
}
// global and constant address-space views of the item's arrays: global loads instead of
// flat ones, and scalar loads for the coefficients
using GU32 = const __attribute__((address_space(1))) uint32_t *;
using GU64 = const __attribute__((address_space(1))) uint64_t *;
using GI64 = const __attribute__((address_space(1))) int64_t *;
using CU64 = const __attribute__((address_space(4))) uint64_t *;

template <int NC, bool E1>
__device__ __forceinline__ void seg16_quads(const BItem &I, uint64_t begin_, uint64_t end_, uint64_t cell0_, int t0_,
                                            int t1_, uint32_t *s_w, unsigned long long *sk_)
{
    const GU32 keys = (GU32)uni(I.keys);
    const GI64 weights = (GI64)uni(I.weights);
    const CU64 coef = (CU64)uni(I.coef);
    const int cpr = (int)uni((uint32_t)I.cpr);
    const uint32_t m = uni(I.m);
    const bool vec2 = uni((uint32_t)I.vec2) != 0;
    const uint64_t begin = uni(begin_), end = uni(end_), cell0 = uni(cell0_);
    const int t0 = (int)uni((uint32_t)t0_), t1 = (int)uni((uint32_t)t1_);
    unsigned long long *sk = uni(sk_);
    const DevPlan plan = I.plan;
    const uint64_t len = end - begin, nq = len >> 2;
    struct Quad {
        uint32_t x[4][NC];
        uint32_t wneg;  // bit g: tuple g's Delta is -1 (16-bit segments take Deltas +-1 only)
    };
    struct Pend {
        uint32_t old, inc, loc;
    };
    auto load1 = [&](uint64_t i, uint32_t (&x)[NC]) {
        if constexpr (NC == 2) {
            if (vec2) {
                const uint64_t v = ((GU64)keys)[i];  // little-endian: column 0 in the low word
                x[0] = (uint32_t)v;
                x[1] = (uint32_t)(v >> 32);
                return;
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = keys[i * NC + c];
    };
    auto load_quad = [&](uint64_t q, Quad &Q) {
        const uint64_t i0 = begin + 4 * q;
        Q.wneg = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            load1(i0 + g, Q.x[g]);
            if (weights) Q.wneg |= (uint32_t)((uint64_t)weights[i0 + g] >> 63) << g;
        }
    };
    auto add1 = [&](uint32_t row, uint32_t j, uint32_t neg) -> Pend {
        if constexpr (E1) j &= m - 1;
        const uint32_t loc = row + j;  // row is a multiple of m, so even
        const uint32_t inc = inc16(neg, (j & 1u) << 4);
        return Pend{atomicAdd(&s_w[loc >> 1], inc), inc, loc};
    };
    auto check = [&](const Pend *P, int k) {
        uint32_t all = 0x80008000u;
        for (int g = 0; g < k; ++g) all &= P[g].old + P[g].inc + 0x40004000u;
        if (all != 0x80008000u) {
            for (int g = 0; g < k; ++g)
                if (out16(P[g].old, P[g].inc)) spill16(&s_w[P[g].loc >> 1], shift16(P[g].inc), sk + cell0 + P[g].loc);
        }
    };
    // hash tuples [0, K) of a quad for repetition t, add them, check them
    auto run = [&](const Quad &Q, auto kc, int t) {
        constexpr int K = decltype(kc)::value;
        const CU64 cf = coef + (size_t)t * cpr;
        const uint32_t row = (uint32_t)((uint64_t)t * m - cell0);
        uint32_t j[K], neg[K];
        if constexpr (E1) {
            CoefE1<NC> C;
            C.load(cf);
            uint32_t flag = 0;
#pragma unroll
            for (int g = 0; g < K; ++g) {
                uint32_t f;
                C.bin_neg_fast(Q.x[g], j[g], neg[g], f);
                flag = max(flag, f);
            }
            if (flag >= 0xFFFFFFFFu) {  // a hash may need the full reduction
#pragma unroll
                for (int g = 0; g < K; ++g) {
                    j[g] = C.bin(Q.x[g]);
                    neg[g] = C.neg(Q.x[g]);
                }
            }
        } else {
#pragma unroll
            for (int g = 0; g < K; ++g) hash_rep<NC>((const uint64_t *)cf, plan, Q.x[g], j[g], neg[g]);
        }
        Pend P[K];
#pragma unroll
        for (int g = 0; g < K; ++g) P[g] = add1(row, j[g], neg[g] ^ ((Q.wneg >> g) & 1u));
        check(P, K);
    };
    if (nq > 0) {
        const uint64_t last = nq - 1;
        uint64_t q = threadIdx.x;
        Quad A, B;
        load_quad(q < last ? q : last, A);
        while (q < nq) {
            load_quad(q + kBBlock < last ? q + kBBlock : last, B);
            for (int t = t0; t <= t1; ++t) run(A, std::integral_constant<int, 4>{}, t);
            q += kBBlock;
            if (q >= nq) break;
            load_quad(q + kBBlock < last ? q + kBBlock : last, A);
            for (int t = t0; t <= t1; ++t) run(B, std::integral_constant<int, 4>{}, t);
            q += kBBlock;
        }
    }
    if ((uint64_t)threadIdx.x < (len & 3)) {
        const uint64_t i = begin + 4 * nq + threadIdx.x;
        Quad Q;
        load1(i, Q.x[0]);
        Q.wneg = weights ? (uint32_t)((uint64_t)weights[i] >> 63) : 0u;
        for (int t = t0; t <= t1; ++t) run(Q, std::integral_constant<int, 1>{}, t);
    }
}

template <int NC>
__device__ void run_segment16(const BItem &I, uint32_t seg, uint64_t begin, uint64_t end, uint32_t *s_w)
{
    const uint64_t cells = (uint64_t)I.d * I.m;
    const uint64_t cell0 = (uint64_t)seg * I.R;
    const uint64_t cell1 = cell0 + I.R < cells ? cell0 + I.R : cells;
    const uint32_t span = (uint32_t)(cell1 - cell0);  // even: R and m are even
    const int t0 = (int)(cell0 / I.m);
    const int t1 = (int)((cell1 - 1) / I.m);
    const bool whole = I.R >= I.m;
    unsigned long long *sk = reinterpret_cast<unsigned long long *>(I.sketch);
    for (uint32_t e = threadIdx.x; e < span / 2; e += kBBlock) s_w[e] = (kBias16 << 16) | kBias16;
    __syncthreads();
    uint64_t i = begin + threadIdx.x;
    uint32_t p_old = kBias16 * 0x10001u, p_inc = 0;  // before the first add: in range
    uint64_t p_g = 0;
    uint32_t *p_w = s_w;
    if constexpr (NC <= 2) {
        if (whole) {
            if (I.e1) seg16_quads<NC, true>(I, begin, end, cell0, t0, t1, s_w, sk);
            else seg16_quads<NC, false>(I, begin, end, cell0, t0, t1, s_w, sk);
            i = end;  // the loop below has nothing left
        }
    }
    uint32_t xn[NC];
    int64_t wn = 0;
    if (i < end) {
        load_keys<NC>(I.keys, i, I.vec2 != 0, xn);
        if (I.weights) wn = I.weights[i];
    }
    for (; i < end; i += kBBlock) {
        uint32_t x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = xn[c];
        const int64_t wt = wn;
        if (i + kBBlock < end) {
            load_keys<NC>(I.keys, i + kBBlock, I.vec2 != 0, xn);
            if (I.weights) wn = I.weights[i + kBBlock];
        }
        for (int t = t0; t <= t1; ++t) {
            const uint64_t *cf = I.coef + (size_t)t * I.cpr;
            uint32_t j, neg;
            if (whole) {
                hash_rep<NC>(cf, I.plan, x, j, neg);
            } else {
                j = hash_bin<NC>(cf, I.plan, x);
                const uint64_t flat = (uint64_t)t * I.m + j;
                if (flat < cell0 || flat >= cell1) continue;
                neg = hash_neg<NC>(cf, I.plan, x);
            }
            if (wt < 0) neg ^= 1u;
            const uint64_t g = (uint64_t)t * I.m + j;
            const uint32_t loc = (uint32_t)(g - cell0);
            uint32_t *w = &s_w[loc >> 1];
            const uint32_t inc = inc16(neg, (loc & 1u) << 4);
            const uint32_t old = atomicAdd(w, inc);
            if (out16(p_old, p_inc)) spill16(p_w, shift16(p_inc), sk + p_g);
            p_old = old;
            p_inc = inc;
            p_g = g;
            p_w = w;
        }
    }
    if (out16(p_old, p_inc)) spill16(p_w, shift16(p_inc), sk + p_g);
    __syncthreads();
    unsigned long long *out = sk + cell0;
    for (uint32_t e = threadIdx.x; e < span / 2; e += kBBlock) {
        const uint32_t w = s_w[e];
        const int64_t lo = (int64_t)(w & 0xFFFFu) - (int64_t)kBias16;
        const int64_t hi = (int64_t)(w >> 16) - (int64_t)kBias16;
        if (lo) atomicAdd(out + 2 * e, (unsigned long long)lo);
        if (hi) atomicAdd(out + 2 * e + 1, (unsigned long long)hi);
    }
    __syncthreads();
}

template <int NC>
__device__ void run_task(const BItem &I, const BTask &T, unsigned char *lds)
{
    if (T.kind == 0) {
        run_atomic<NC>(I, T.begin, T.end);
    } else if (T.kind == 2) {
        run_sortreduce<NC>(I, T.begin, T.end);
    } else if (I.narrow) {
        run_segment16<NC>(I, T.seg, T.begin, T.end, reinterpret_cast<uint32_t *>(lds));
    } else {
        run_segment<NC, int64_t>(I, T.seg, T.begin, T.end, reinterpret_cast<int64_t *>(lds));
    }
}

// Persistent workgroups pull tasks until the list is exhausted; every workgroup exits
// once the shared counter passes n_tasks.
__global__ __launch_bounds__(kBBlock) void k_batch_update(const BItem *__restrict__ items,
                                                          const BTask *__restrict__ tasks, int32_t n_tasks,
                                                          unsigned int *counter)
{
    extern __shared__ __align__(16) unsigned char s_lds[];
    __shared__ int s_task;
    for (;;) {
        if (threadIdx.x == 0) s_task = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // wave-uniform, so the task and item fields load into scalar registers
        const int task = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();
        if (task >= n_tasks) break;
        const BTask T = tasks[task];
        const BItem I = items[T.item];
        switch (I.n_cols) {
            case 1: run_task<1>(I, T, s_lds); break;
            case 2: run_task<2>(I, T, s_lds); break;
            case 3: run_task<3>(I, T, s_lds); break;
            case 4: run_task<4>(I, T, s_lds); break;
            case 5: run_task<5>(I, T, s_lds); break;
            case 6: run_task<6>(I, T, s_lds); break;
            case 7: run_task<7>(I, T, s_lds); break;
            default: run_task<8>(I, T, s_lds); break;
        }
    }
}

__global__ void k_batch_zero(uint64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_batch_diff(const uint64_t *__restrict__ x, const uint64_t *__restrict__ y, size_t n,
                             unsigned int *flag)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (x[i] != y[i]) atomicOr(flag, 1u);
}

}  // namespace

// Host side of a batch: work-list planning, device tables, optional graph.
struct BatchState {
    int device = -1;
    void *tables = nullptr;    // items, tasks, counter
    size_t table_bytes = 0;
    int32_t n_tasks = 0;
    size_t o_items = 0, o_tasks = 0, o_counter = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    EstimateWork est;
    std::vector<Handle *> est_handles;
    uint64_t tasks_atomic = 0, tasks_segment = 0, tasks_sort = 0;
};

namespace {

// One item's table entry and what its task planning needs.
struct ItemInfo {
    BItem I;
    int steps;         // Horner steps per tuple and repetition
    int e1, unit;
};

cs_status make_item(const cs_update_item &it, BItem &I, ItemInfo &info)
{
    const Handle &h = it.sketch->h;
    const RelPlan &rp = h.g.rel[it.rel];
    cs_status chk = check_device_array(it.keys, it.n * rp.n_cols * sizeof(uint32_t), h.device, "batch keys");
    if (chk == CS_OK && it.weights) chk = check_device_array(it.weights, it.n * sizeof(int64_t), h.device, "batch weights");
    if (chk != CS_OK) return chk;
    I = BItem{};
    I.keys = it.keys;
    I.weights = it.weights;
    I.coef = h.coef_dev + h.coef_off[it.rel];
    I.sketch = reinterpret_cast<uint64_t *>(h.counters + (size_t)it.rel * h.d * h.m);
    I.n = it.n;
    I.cpr = rp.coef_per_rep;
    I.n_cols = rp.n_cols;
    I.m = h.m;
    I.log2m = h.log2m;
    I.d = (int32_t)h.d;
    const bool unit = it.weights == nullptr || (it.flags & CS_UPDATE_UNIT_WEIGHTS);
    I.narrow = unit && it.n < (1ull << 31) && (h.m % 2) == 0;  // 16-bit pairs need even segments
    I.vec2 = rp.n_cols == 2 && ((uintptr_t)it.keys % 8) == 0;
    for (int c = 0; c < kMaxCols; ++c) I.plan.n_edges[c] = c < rp.n_cols ? rp.n_edges[c] : 0;
    I.plan.bm = make_binmod(h.m);
    I.e1 = (h.m & (h.m - 1)) == 0;
    for (int c = 0; c < rp.n_cols; ++c) I.e1 = I.e1 && rp.n_edges[c] == 1;
    // LDS segment: 2^16 16-bit counters (Deltas +-1) or 2^14 int64 counters
    uint32_t R = I.narrow ? (1u << 16) : (1u << 14);
    if (h.m <= R) R = (R / h.m) * h.m;
    I.R = R;
    info.I = I;
    info.steps = 0;
    for (int c = 0; c < rp.n_cols; ++c) info.steps += 1 + 3 * rp.n_edges[c];
    info.e1 = 1;
    for (int c = 0; c < rp.n_cols; ++c) info.e1 = info.e1 && rp.n_edges[c] == 1;
    info.unit = unit ? 1 : 0;
    return CS_OK;
}

// The fixed rule: global atomics where aggregation cannot pay (a few microseconds of
// them at most; a segment task's fixed cost is zeroing and flushing its LDS counters),
// else LDS segments over tuple chunks of at most 2^18 (chunk_log2 -1: balanced chunks).
void rule_choice(const BItem &I, int *kind, int *chunk_log2)
{
    const uint64_t cells = (uint64_t)I.d * I.m;
    const uint64_t tuple_reps = I.n * I.d;
    if (tuple_reps < 65536 || tuple_reps < cells / 4) {
        *kind = 0;
        *chunk_log2 = 16;
    } else {
        *kind = 1;
        *chunk_log2 = -1;
    }
}

// Tasks of item idx with the given kind and tuple chunk (2^chunk_log2, or for -1 the
// balanced chunks of at most 2^18).
void add_tasks(int idx, const ItemInfo &info, int kind, int chunk_log2, std::vector<BTask> &bt,
               std::vector<double> &cost, uint64_t &n_atomic, uint64_t &n_segment, uint64_t &n_sort)
{
    const BItem &I = info.I;
    const uint64_t n = I.n;
    const uint64_t cells = (uint64_t)I.d * I.m;
    uint64_t chunk;
    if (chunk_log2 < 0) {
        const uint64_t C = (n + (1u << 18) - 1) >> 18;
        chunk = (n + C - 1) / C;
    } else {
        const uint64_t C = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
        chunk = (n + C - 1) / C;
    }
    if (kind == 0 || kind == 2) {
        // sort-reduce: the exchange network (21 steps of a key and a 64-bit value) per
        // tuple and repetition in place of most of the atomics
        const double per = kind == 0 ? info.steps + 40 : info.steps + 160;
        for (uint64_t b = 0; b < n; b += chunk) {
            BTask T{idx, kind, 0, 0, b, std::min<uint64_t>(n, b + chunk)};
            bt.push_back(T);
            cost.push_back((double)(T.end - T.begin) * I.d * per);
            ++(kind == 0 ? n_atomic : n_sort);
        }
    } else {
        const uint32_t R = I.R;
        const uint32_t segs = (uint32_t)((cells + R - 1) / R);
        const int reps_per_seg = R >= I.m ? (int)(R / I.m) : 1;
        const int ranges = R >= I.m ? 1 : (int)(I.m / R);
        for (uint32_t sg = 0; sg < segs; ++sg)
            for (uint64_t b = 0; b < n; b += chunk) {
                BTask T{idx, 1, sg, 0, b, std::min<uint64_t>(n, b + chunk)};
                bt.push_back(T);
                cost.push_back((double)(T.end - T.begin) * reps_per_seg * (info.steps + ranges) + R);
                ++n_segment;
            }
    }
}

// Sorts the tasks largest first and uploads items and tasks.
cs_status upload_tables(BatchState &B, const std::vector<BItem> &bi, const std::vector<BTask> &bt,
                        const std::vector<double> &cost, hipStream_t s)
{
    std::vector<int> order(bt.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<BTask> sorted(bt.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = bt[order[i]];
    const size_t o_items = 0;
    const size_t o_tasks = (bi.size() * sizeof(BItem) + 255) & ~(size_t)255;
    const size_t o_counter = o_tasks + ((sorted.size() * sizeof(BTask) + 255) & ~(size_t)255);
    const size_t bytes = o_counter + 256;
    if (B.table_bytes < bytes) {
        if (B.tables) {
            CSK_HIP(hipStreamSynchronize(s));
            hipFree(B.tables);
        }
        B.tables = nullptr;
        B.table_bytes = 0;
        if (hipMalloc(&B.tables, bytes) != hipSuccess) return fail(CS_ENOMEM, "batch tables");
        B.table_bytes = bytes;
    }
    std::vector<char> img(o_counter, 0);
    if (!bi.empty()) std::memcpy(img.data() + o_items, bi.data(), bi.size() * sizeof(BItem));
    if (!sorted.empty()) std::memcpy(img.data() + o_tasks, sorted.data(), sorted.size() * sizeof(BTask));
    CSK_HIP(hipMemcpyAsync(B.tables, img.data(), img.size(), hipMemcpyHostToDevice, s));
    CSK_HIP(hipStreamSynchronize(s));
    B.n_tasks = (int32_t)sorted.size();
    B.o_items = o_items;
    B.o_tasks = o_tasks;
    B.o_counter = o_counter;
    return CS_OK;
}

cs_status plan_batch(BatchState &B, const cs_update_item *items, int32_t n_items, hipStream_t s)
{
    std::vector<BItem> bi;
    std::vector<BTask> bt;
    std::vector<double> cost;
    B.tasks_atomic = B.tasks_segment = B.tasks_sort = 0;
    for (int32_t i = 0; i < n_items; ++i) {
        const cs_update_item &it = items[i];
        if (!it.sketch) return fail(CS_EINVAL, "batch item without handle");
        const Handle &h = it.sketch->h;
        if (it.rel < 0 || it.rel >= h.g.n_rel) return fail(CS_EINVAL, "batch item relation out of range");
        if (it.n == 0) continue;
        if (!it.keys) return fail(CS_EINVAL, "batch item without keys");
        if (B.device < 0) B.device = h.device;
        if (h.device != B.device) return fail(CS_EINVAL, "batch items on different devices");
        BItem I;
        ItemInfo info;
        cs_status st = make_item(it, I, info);
        if (st != CS_OK) return st;
        int kind, chunk_log2;
        if (!tune_lookup_batch(h.device, h.m, (int)h.d, I.n_cols, info.e1, info.unit, it.n, &kind, &chunk_log2))
            rule_choice(I, &kind, &chunk_log2);
        const int idx = (int)bi.size();
        bi.push_back(I);
        add_tasks(idx, info, kind, chunk_log2, bt, cost, B.tasks_atomic, B.tasks_segment, B.tasks_sort);
    }
    return upload_tables(B, bi, bt, cost, s);
}

cs_status launch_batch(BatchState &B, hipStream_t s)
{
    if (B.n_tasks == 0) return CS_OK;
    char *t = static_cast<char *>(B.tables);
    unsigned int *counter = reinterpret_cast<unsigned int *>(t + B.o_counter);
    int n_cu = 256;
    CSK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, B.device));
    const int grid = std::min(n_cu, B.n_tasks);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
    CSK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_batch_update, dim3(grid), dim3(kBBlock), kBLds, s,
                       reinterpret_cast<const BItem *>(t + B.o_items), reinterpret_cast<const BTask *>(t + B.o_tasks),
                       B.n_tasks, counter);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

void drop_graph(BatchState &B)
{
    if (B.exec) hipGraphExecDestroy(B.exec);
    if (B.graph) hipGraphDestroy(B.graph);
    B.exec = nullptr;
    B.graph = nullptr;
}

}  // namespace

}  // namespace csk

using namespace csk;

struct cs_batch {
    BatchState b;
};

extern "C" {

cs_status cs_batch_create(cs_batch **out)
{
    if (!out) return fail(CS_EINVAL, "null output");
    cs_batch *b = new (std::nothrow) cs_batch();
    if (!b) return fail(CS_ENOMEM, "host allocation failed");
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_update),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBLds));
    *out = b;
    return CS_OK;
}

cs_status cs_batch_destroy(cs_batch *b)
{
    if (!b) return CS_OK;
    hipDeviceSynchronize();
    drop_graph(b->b);
    if (b->b.capture_stream) hipStreamDestroy(b->b.capture_stream);
    if (b->b.tables) hipFree(b->b.tables);
    release_work(b->b.est);
    delete b;
    return CS_OK;
}

cs_status cs_batch_update(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream)
{
    if (!b || (n_items > 0 && !items)) return fail(CS_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    cs_status st = plan_batch(b->b, items, n_items, s);
    if (st != CS_OK) return st;
    return launch_batch(b->b, s);
}

cs_status cs_batch_capture(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream)
{
    if (!b || (n_items > 0 && !items)) return fail(CS_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    drop_graph(b->b);
    cs_status st = plan_batch(b->b, items, n_items, s);
    if (st != CS_OK) return st;
    // capture on a private stream (the null stream cannot be captured); the graph is
    // launched later on the caller's stream
    if (!b->b.capture_stream) CSK_HIP(hipStreamCreateWithFlags(&b->b.capture_stream, hipStreamNonBlocking));
    hipStream_t cs = b->b.capture_stream;
    CSK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    st = launch_batch(b->b, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != CS_OK) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->b.graph = g;
    CSK_HIP(hipGraphInstantiate(&b->b.exec, g, nullptr, nullptr, 0));
    return CS_OK;
}

cs_status cs_batch_replay(cs_batch *b, void *stream)
{
    if (!b || !b->b.exec) return fail(CS_EINVAL, "no captured batch");
    CSK_HIP(hipGraphLaunch(b->b.exec, static_cast<hipStream_t>(stream)));
    return CS_OK;
}

cs_status cs_batch_estimate(cs_batch *b, cs_sketch *const *sketches, int32_t n, void *stream, cs_estimate_t *outs,
                            const cs_reps_t *reps)
{
    if (!b || (n > 0 && (!sketches || !outs))) return fail(CS_EINVAL, "null argument");
    std::vector<Handle *> hs(n);
    for (int i = 0; i < n; ++i) {
        if (!sketches[i]) return fail(CS_EINVAL, "null handle in batch");
        hs[i] = &sketches[i]->h;
    }
    return estimate_batch(hs.data(), n, static_cast<hipStream_t>(stream), outs, reps, b->b.est);
}

cs_status cs_batch_stats(const cs_batch *b, uint64_t *tasks_atomic, uint64_t *tasks_segment)
{
    if (!b) return fail(CS_EINVAL, "null batch");
    if (tasks_atomic) *tasks_atomic = b->b.tasks_atomic;
    if (tasks_segment) *tasks_segment = b->b.tasks_segment;
    return CS_OK;
}

cs_status cs_batch_task_counts(const cs_batch *b, uint64_t *tasks_atomic, uint64_t *tasks_segment,
                               uint64_t *tasks_sort_reduce)
{
    if (!b) return fail(CS_EINVAL, "null batch");
    if (tasks_atomic) *tasks_atomic = b->b.tasks_atomic;
    if (tasks_segment) *tasks_segment = b->b.tasks_segment;
    if (tasks_sort_reduce) *tasks_sort_reduce = b->b.tasks_sort;
    return CS_OK;
}

cs_status cs_tune_batch_update(cs_batch *b, const cs_update_item *items, int32_t n_items, void *stream,
                               cs_tune_batch_report *out)
{
    if (!b || !out || (n_items > 0 && !items)) return fail(CS_EINVAL, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::memset(out, 0, sizeof(*out));
    // classes: (m, d, key columns, one-join columns, unit weights, floor(log2 n))
    using Key = std::tuple<uint32_t, int, int, int, int, int>;
    std::map<Key, std::vector<int>> classes;
    std::vector<ItemInfo> info(n_items);
    int device = -1;
    for (int32_t i = 0; i < n_items; ++i) {
        const cs_update_item &it = items[i];
        if (!it.sketch) return fail(CS_EINVAL, "batch item without handle");
        const Handle &h = it.sketch->h;
        if (it.rel < 0 || it.rel >= h.g.n_rel) return fail(CS_EINVAL, "batch item relation out of range");
        if (it.n == 0) continue;
        if (!it.keys) return fail(CS_EINVAL, "batch item without keys");
        if (device < 0) device = h.device;
        if (h.device != device) return fail(CS_EINVAL, "batch items on different devices");
        BItem I;
        cs_status st = make_item(it, I, info[i]);
        if (st != CS_OK) return st;
        int lg = 0;
        while ((it.n >> (lg + 1)) != 0) ++lg;
        classes[Key{h.m, (int)h.d, I.n_cols, info[i].e1, info[i].unit, lg}].push_back(i);
    }
    if (classes.empty()) return CS_OK;
    size_t max_cells = 0;
    for (auto &kv : classes) {
        size_t c = 0;
        for (int i : kv.second) c += (size_t)info[i].I.d * info[i].I.m;
        max_cells = std::max(max_cells, c);
    }
    uint64_t *ref = nullptr, *tmp = nullptr, *rep = nullptr;
    // replicas of a class for timing: up to 64 copies, at most 1 GiB
    const size_t rep_cells = std::max<size_t>(max_cells, std::min<size_t>(64 * max_cells, ((size_t)1 << 30) / 8));
    unsigned int *flag = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BatchState T;
    T.device = device;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (ref) (void)hipFree(ref);
        if (tmp) (void)hipFree(tmp);
        if (rep) (void)hipFree(rep);
        if (flag) (void)hipFree(flag);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (T.tables) (void)hipFree(T.tables);
    };
    if (hipMalloc(&ref, max_cells * 8) != hipSuccess || hipMalloc(&tmp, max_cells * 8) != hipSuccess ||
        hipMalloc(&rep, rep_cells * 8) != hipSuccess ||
        hipMalloc(&flag, sizeof(unsigned int)) != hipSuccess) {
        cleanup();
        return fail(CS_ENOMEM, "batch tuning buffers");
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(CS_EDEVICE, "batch tuning events");
    }
    // candidates: (kind, log2 tuples per task); index 0, global atomics, is the reference;
    // index 1 is the fixed rule (measured for the report, never stored); kind 2 is
    // sort-reduce, kind 1 LDS segments
    const int cands[][2] = {{0, 16}, {-1, -1}, {2, 16}, {1, 14}, {1, 16}, {1, 18}, {1, 20}};
    const int n_cand = (int)(sizeof(cands) / sizeof(cands[0]));
    cs_status st = CS_OK;
    for (auto &kv : classes) {
        const std::vector<int> &members = kv.second;
        size_t cells = 0;
        std::vector<size_t> off;
        for (int i : members) {
            off.push_back(cells);
            cells += (size_t)info[i].I.d * info[i].I.m;
        }
        const unsigned zb = (unsigned)std::min<size_t>((cells + 255) / 256, 4096);
        float best_ms = -1.0f, rule_ms = -1.0f;
        int best_kind = 0, best_chunk = 16;
        for (int ci = 0; ci < n_cand && st == CS_OK; ++ci) {
            // the class's items with this candidate's tasks, `copies` times over, copy c
            // adding into dst + c * cells
            auto build = [&](uint64_t *dst, int copies) {
                std::vector<BItem> bi;
                std::vector<BTask> bt;
                std::vector<double> cost;
                uint64_t na = 0, ns = 0, nr = 0;
                for (int c = 0; c < copies; ++c)
                    for (size_t j = 0; j < members.size(); ++j) {
                        ItemInfo ii = info[members[j]];
                        ii.I.sketch = dst + (size_t)c * cells + off[j];
                        int kind = cands[ci][0], chunk = cands[ci][1];
                        if (kind < 0) rule_choice(ii.I, &kind, &chunk);
                        const int idx = (int)bi.size();
                        bi.push_back(ii.I);
                        add_tasks(idx, ii, kind, chunk, bt, cost, na, ns, nr);
                    }
                return upload_tables(T, bi, bt, cost, s);
            };
            uint64_t *dst = ci == 0 ? ref : tmp;
            if ((st = build(dst, 1)) != CS_OK) break;
            hipLaunchKernelGGL(k_batch_zero, dim3(zb), dim3(256), 0, s, dst, cells);
            if ((st = launch_batch(T, s)) != CS_OK) break;
            if (ci > 0) {
                unsigned int hflag = 0;
                hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, flag);
                hipLaunchKernelGGL(k_batch_diff, dim3(zb), dim3(256), 0, s, tmp, ref, cells, flag);
                if (hipMemcpyAsync(&hflag, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st = fail(CS_EDEVICE, "batch tuning: compare");
                    break;
                }
                if (hflag) {  // counters differ from the reference: never chosen
                    out->rejected++;
                    continue;
                }
            }
            // timed: median of three runs of enough copies of the class's work to fill the
            // chip (its cost inside a large batch is its throughput, not the latency of a
            // launch of it alone), each copy adding into its own counters (never into the
            // reference, which later candidates are checked against)
            const int copies = (int)std::max<int64_t>(
                1, std::min<int64_t>({(2048 + T.n_tasks - 1) / std::max<int32_t>(1, T.n_tasks), 64,
                                      (int64_t)(rep_cells / std::max<size_t>(1, cells))}));
            if ((st = build(rep, copies)) != CS_OK) break;
            float t[3];
            bool ok = true;
            for (int r = 0; r < 3 && ok; ++r)
                ok = hipEventRecord(e0, s) == hipSuccess && launch_batch(T, s) == CS_OK &&
                     hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
            if (!ok) {
                st = fail(CS_EDEVICE, "batch tuning: timing");
                break;
            }
            std::sort(t, t + 3);
            t[1] /= (float)copies;
            if (ci == 1) {
                rule_ms = t[1];
                continue;
            }
            if (best_ms < 0.0f || t[1] < best_ms) {
                best_ms = t[1];
                best_kind = cands[ci][0];
                best_chunk = cands[ci][1];
            }
        }
        if (st != CS_OK) break;
        const Key &k = kv.first;
        const ItemInfo &i0 = info[members[0]];
        tune_store_batch(device, std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                         i0.I.n, best_kind, best_chunk, best_ms);
        out->classes++;
        out->rule_ms += rule_ms < 0.0f ? best_ms : rule_ms;
        out->tuned_ms += best_ms;
    }
    cleanup();
    return st;
}

}  // extern "C"
