// Sketches of the sub-queries a query optimizer evaluates, built in one pass over each
// relation (Sec. 3.4).
//
// An optimizer enumerating join orders needs the size of many sub-queries of one base
// query: each sub-query is a connected subset of the base query's joins.  Every
// relation of a sub-query needs a Count sketch built with that sub-query's hash
// functions, and the same relation appears in many sub-queries.  The hash functions are
// assigned so that sketches coincide wherever the paper allows reuse:
//   * bin hash of an attribute: one degree-1 polynomial per base component (per
//     repetition), whatever sub-query the attribute is in;
//   * sign hash of a join: when the join is the only join of its component inside the
//     sub-query, the component's shared degree-3 polynomial, so an attribute's sketch
//     is the same for every sub-query that joins it once; when the component holds two
//     or more of the sub-query's joins, each join takes its own polynomial (an attribute
//     joined twice inside one sub-query needs two independent signs: the shared
//     polynomial multiplied by itself would be 1).
// A relation's sketch in a sub-query is therefore fixed by which of its columns are
// joined there and by the sign polynomials of each; the distinct ones are the targets,
// each an int64 [d][m] sketch, and a sub-query's estimate reads its relations' targets.
//
// Update (Alg. 2 for every target of a relation, one read of its keys): pass 1 hashes
// each (tuple, repetition) once — the bin value of every column and the sign bit of
// every (column, polynomial) any target uses — and every target combines them (sum of
// its columns' bins mod m, parity of its sign bits) into a 16-bit record (14-bit offset
// in a 2^14-bucket range, sign bit), ranked per bucket range in LDS and staged per block
// in runs padded to four records.  Pass 2: one workgroup per (range, target,
// repetition) sums the runs of every block in LDS and adds the sums into the counters
// it alone owns.  Deltas must be +1 (weights NULL) or +-1 (CS_UPDATE_UNIT_WEIGHTS);
// general weights take one global atomic per (tuple, target, repetition).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "csk_handle.h"
#include "csk_hash.h"
#include "csk_internal.h"

namespace csk {

constexpr int kSqMaxCols = 4;        // key columns of a base relation
constexpr int kSqMaxTargets = 16;    // distinct sketches of one relation
constexpr int kSqMaxSign = 16;       // distinct (column, sign polynomial) pairs of one relation
constexpr int kSqMaxSub = 4096;      // sub-queries of one handle

// What pass 1 needs of one relation: per column the range of its sign evaluations, per
// target the columns whose bins it sums and the sign evaluations whose bits it XORs.
struct SqDesc {
    int32_t nt, ns;
    int32_t s_beg[kSqMaxCols + 1];
    uint32_t col_mask[kSqMaxTargets];
    uint32_t sign_mask[kSqMaxTargets];
};
struct SqTargets {
    uint64_t *p[kSqMaxTargets];  // counters [d][m] of each target of the relation
};

struct SqRel {
    int a = 0;                                // key columns (the base relation's attributes)
    std::vector<std::pair<int, int>> sev;     // (column, sign polynomial id), by column
    std::vector<int> targets;                 // global target ids, in the relation's order
    std::vector<uint32_t> col_mask, sign_mask;
    uint64_t *coef_dev = nullptr;             // [d][2 a + 4 |sev|]
    int cpr = 0;
};

struct SqTarget {
    int rel = 0;
    std::vector<std::pair<int, std::vector<int>>> cols;  // (column, sign polynomial ids)
};

struct SqQuery {
    uint32_t mask = 0;
    std::vector<int> rels;     // base relations, ascending
    Handle view;               // the induced query's plan, counters taken from the targets
};

struct SubqHandle {
    int device = 0;
    uint32_t m = 0, d = 0;
    uint64_t seed = 0;
    GraphPlan g;
    std::vector<uint64_t> comp_sign;  // [d][Q][4]
    std::vector<uint64_t> bin;        // [d][Q][2]
    std::vector<uint64_t> edge_sign;  // [d][E][4]
    std::vector<SqRel> rel;
    std::vector<SqTarget> targets;
    std::vector<SqQuery> sub;
    int64_t *counters = nullptr;      // [targets][d][m]
    void *scratch = nullptr;          // pass-1 records and run tables of one chunk
    size_t scratch_bytes = 0;
    uint64_t chunk_blocks = 0;        // pass-1 blocks per chunk
    EstimateWork est;                 // workspace of cs_subq_estimate_all
};

}  // namespace csk

struct cs_subq {
    csk::SubqHandle h;
};

namespace csk {
namespace {

constexpr int kSqB = 256;                     // pass-1 workgroup
constexpr int kSqSlots = 8;                   // tuples per thread
constexpr int kSqBlk = kSqB * kSqSlots;       // 2048 tuples per block
constexpr int kSqLog2R = 14;                  // buckets per range
constexpr uint32_t kSqR = 1u << kSqLog2R;
constexpr int kSqHS = 4;                      // sub-histograms per range (lane & 3)
constexpr int kSqCap = kSqBlk + 4 * 64;       // a block's records of one (target, repetition)
constexpr int kSqAB = 1024;                   // pass-2 workgroup
constexpr uint32_t kSqNone = 0xFFFFFFFFu;
constexpr uint16_t kSqPad = 0xFFFFu;          // padding record (bit 15 set: never a real one)
constexpr size_t kSqScratchBudget = 256ull << 20;
static_assert(kSqCap % 8 == 0 && kSqCap <= 0xFFFF, "16-byte stores, 16-bit run starts");
static_assert(kMaxLog2M - kSqLog2R <= 6, "at most 64 ranges");

__device__ __forceinline__ void sq_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pass 1.  Grid (blocks, repetition groups) mapped by seg_tile(): the groups of one
// block run on one XCD, whose L2 fetches the block's keys once.
template <int NC, bool HW>
__global__ __launch_bounds__(kSqB) void k_subq_hash(const uint32_t *__restrict__ keys,
                                                    const int64_t *__restrict__ weights, uint64_t n,
                                                    const uint64_t *__restrict__ coef, int32_t cpr, SqDesc D,
                                                    BinMod bm, int32_t d, int32_t ranges, int32_t reps_per_group,
                                                    uint64_t nblk, uint16_t *rec, uint16_t *tab)
{
    __shared__ __align__(16) uint32_t s_hist[kSqB / 64][64 * kSqHS];
    __shared__ uint32_t s_tot[kSqB / 64][64];
    __shared__ __align__(16) uint16_t s_stage[kSqCap];
    const SegTile wg = seg_tile();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t blk = wg.chunk;
    const int t0 = (int)wg.seg * reps_per_group;
    const int t1 = min(d, t0 + reps_per_group);

    // slot s holds tuple blk * kSqBlk + s * kSqB + threadIdx.x (coalesced loads)
    uint32_t x[kSqSlots][NC];
    uint32_t valid = 0, wneg = 0;
#pragma unroll
    for (int s = 0; s < kSqSlots; ++s) {
        const uint64_t i = blk * kSqBlk + (uint64_t)s * kSqB + threadIdx.x;
        const bool in = i < n;
        const uint64_t ic = in ? i : 0;  // clamped: every load stays in bounds
#pragma unroll
        for (int c = 0; c < NC; ++c) x[s][c] = keys[ic * NC + c];
        if constexpr (HW) wneg |= (uint32_t)((uint64_t)weights[ic] >> 63) << s;
        valid |= (uint32_t)in << s;
    }
    wneg &= valid;

    uint32_t *hist = s_hist[wave];
    const uint32_t sub = lane & (kSqHS - 1);
    for (int t = t0; t < t1; ++t) {
        const uint64_t *cf = coef + (size_t)t * cpr;
        // the column bins (canonical, below p) and one sign bit per evaluation
        uint64_t bv[kSqSlots][NC];
        uint32_t sb[kSqSlots];
#pragma unroll
        for (int s = 0; s < kSqSlots; ++s) {
            sb[s] = 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) bv[s][c] = hash_deg1(cf + 2 * c, x[s][c]);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            for (int e = D.s_beg[c]; e < D.s_beg[c + 1]; ++e) {
                const uint64_t *a = cf + 2 * NC + 4 * e;
#pragma unroll
                for (int s = 0; s < kSqSlots; ++s) sb[s] |= ((uint32_t)hash_deg3(a, x[s][c]) & 1u) << e;
            }
        }
        for (int i = 0; i < D.nt; ++i) {
            const uint32_t cm = D.col_mask[i], sm = D.sign_mask[i];
            reinterpret_cast<uint4 *>(hist)[lane] = make_uint4(0u, 0u, 0u, 0u);
            sq_wave_sync();
            uint32_t P[kSqSlots];
#pragma unroll
            for (int s = 0; s < kSqSlots; ++s) {
                P[s] = kSqNone;
                if ((valid >> s) & 1u) {
                    uint64_t js = 0;
#pragma unroll
                    for (int c = 0; c < NC; ++c) js += ((cm >> c) & 1u) ? bv[s][c] : 0ull;
                    const uint32_t b = bm.reduce(js);
                    const uint32_t ng = ((uint32_t)__popc(sb[s] & sm) ^ (wneg >> s)) & 1u;
                    const uint32_t r = b >> kSqLog2R;
                    const uint32_t rc = (b & (kSqR - 1)) | (ng << kSqLog2R);
                    const uint32_t pos = atomicAdd(&hist[r * kSqHS + sub], 1u);  // < 16 * kSqSlots
                    P[s] = rc | (r << 15) | (pos << 21);
                }
            }
            sq_wave_sync();
            // run of range L = lane: this wavefront's four sub-counts and their prefix, the
            // totals of every wavefront; runs padded to multiples of four records
            const uint4 h4 = reinterpret_cast<const uint4 *>(hist)[lane];
            const uint32_t e1 = h4.x, e2 = e1 + h4.y, e3 = e2 + h4.z, tot = e3 + h4.w;
            s_tot[wave][lane] = tot;
            __syncthreads();
            uint32_t before = 0, rtot = 0;
#pragma unroll
            for (int w = 0; w < kSqB / 64; ++w) {
                const uint32_t v = s_tot[w][lane];
                before += w < wave ? v : 0u;
                rtot += v;
            }
            const uint32_t padded = (rtot + 3u) & ~3u;
            uint32_t incl = padded;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            const uint32_t start = incl - padded;
            const uint32_t wb = start + before;
            reinterpret_cast<uint4 *>(hist)[lane] = make_uint4(wb, wb + e1, wb + e2, wb + e3);
            const uint32_t total = __shfl(incl, 63, 64);
            const uint64_t slab = (uint64_t)i * d + t;
            if (wave == 0) {
                uint16_t *tb = tab + (slab * nblk + blk) * (uint64_t)(ranges + 1);
                if (lane < ranges) tb[lane] = (uint16_t)start;
                if (lane == 0) tb[ranges] = (uint16_t)total;
                for (uint32_t e = start + rtot; e < start + padded; ++e) s_stage[e] = kSqPad;
            }
            sq_wave_sync();
#pragma unroll
            for (int s = 0; s < kSqSlots; ++s) {
                if (P[s] != kSqNone) {
                    const uint32_t r = (P[s] >> 15) & 63u;
                    s_stage[hist[r * kSqHS + sub] + (P[s] >> 21)] = (uint16_t)(P[s] & 0x7FFFu);
                }
            }
            __syncthreads();
            uint4 *dst = reinterpret_cast<uint4 *>(rec + (slab * nblk + blk) * kSqCap);
            const uint4 *src = reinterpret_cast<const uint4 *>(s_stage);
            for (uint32_t v = threadIdx.x; v * 8 < total; v += kSqB) dst[v] = src[v];
            __syncthreads();
        }
    }
}

// Pass 2.  Block (range r, slab = target * d + repetition): two copies of 2^14 int32
// LDS counters (even and odd lanes), every block's run of this range added, the sums
// added into the counters this workgroup alone owns.
__global__ __launch_bounds__(kSqAB) void k_subq_accum(const uint16_t *__restrict__ rec,
                                                      const uint16_t *__restrict__ tab, uint64_t nblk,
                                                      int32_t ranges, uint32_t m, int32_t d, SqTargets T)
{
    extern __shared__ __align__(16) uint32_t s_dyn[];
    int32_t *s_cnt = reinterpret_cast<int32_t *>(s_dyn);  // [2][kSqR]
    uint32_t *s_run = s_dyn + 2 * kSqR;                    // [nblk]: start / 4 | words << 16
    const int r = blockIdx.x;
    const uint64_t slab = blockIdx.y;
    const int i = (int)(slab / d), t = (int)(slab % d);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t *my_cnt = s_cnt + (lane & 1) * kSqR;
    constexpr int kWaves = kSqAB / 64;
    constexpr int kInFlight = 4;
    for (uint32_t e = threadIdx.x; e < 2 * kSqR / 4; e += kSqAB) reinterpret_cast<int4 *>(s_cnt)[e] = make_int4(0, 0, 0, 0);
    for (uint64_t b = threadIdx.x; b < nblk; b += kSqAB) {
        const uint16_t *tb = tab + (slab * nblk + b) * (uint64_t)(ranges + 1);
        const uint32_t beg = tb[r], end = tb[r + 1];
        s_run[b] = (beg >> 2) | (((end - beg) >> 2) << 16);
    }
    __syncthreads();
    auto add4 = [&](uint2 w) {
        const uint32_t v[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (v[k] != kSqPad) atomicAdd(&my_cnt[v[k] & (kSqR - 1)], (v[k] >> kSqLog2R) & 1u ? -1 : 1);
    };
    const uint2 *rt = reinterpret_cast<const uint2 *>(rec + slab * nblk * kSqCap);
    for (uint64_t b0 = wave; b0 < nblk; b0 += (uint64_t)kWaves * kInFlight) {
        uint32_t run[kInFlight];
        const uint2 *p[kInFlight];
        uint32_t lmax = 0;
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const uint64_t b = b0 + (uint64_t)u * kWaves;
            run[u] = b < nblk ? s_run[b] : 0u;
            p[u] = rt + (b < nblk ? b : 0) * (kSqCap / 4) + (run[u] & 0xFFFFu);
            lmax = max(lmax, run[u] >> 16);
        }
        for (uint32_t k = lane; k < lmax; k += 64) {
            uint2 w[kInFlight];
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) w[u] = k < (run[u] >> 16) ? p[u][k] : make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
#pragma unroll
            for (int u = 0; u < kInFlight; ++u) add4(w[u]);
        }
    }
    __syncthreads();
    uint64_t *out = T.p[i] + (uint64_t)t * m + ((uint64_t)r << kSqLog2R);
    const uint32_t span = min(kSqR, m - ((uint32_t)r << kSqLog2R));  // the last range may be partial
    for (uint32_t e = threadIdx.x; e < span; e += kSqAB) {
        const int64_t v = (int64_t)s_cnt[e] + (int64_t)s_cnt[kSqR + e];
        if (v) out[e] += (uint64_t)v;
    }
}

// General weights: one global atomic per (tuple, target, repetition).
template <int NC>
__global__ __launch_bounds__(256) void k_subq_atomic(const uint32_t *__restrict__ keys,
                                                     const int64_t *__restrict__ weights, uint64_t n,
                                                     const uint64_t *__restrict__ coef, int32_t cpr, SqDesc D,
                                                     BinMod bm, int32_t d, SqTargets T)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t x[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = keys[i * NC + c];
        const int64_t delta = weights ? weights[i] : 1;
        for (int t = 0; t < d; ++t) {
            const uint64_t *cf = coef + (size_t)t * cpr;
            uint64_t bv[NC];
            uint32_t sb = 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                bv[c] = hash_deg1(cf + 2 * c, x[c]);
                for (int e = D.s_beg[c]; e < D.s_beg[c + 1]; ++e)
                    sb |= ((uint32_t)hash_deg3(cf + 2 * NC + 4 * e, x[c]) & 1u) << e;
            }
            for (int k = 0; k < D.nt; ++k) {
                uint64_t js = 0;
#pragma unroll
                for (int c = 0; c < NC; ++c) js += ((D.col_mask[k] >> c) & 1u) ? bv[c] : 0ull;
                const uint32_t j = bm.reduce(js);
                const bool neg = __popc(sb & D.sign_mask[k]) & 1;
                const uint64_t val = neg ? (uint64_t)0 - (uint64_t)delta : (uint64_t)delta;
                atomicAdd(reinterpret_cast<unsigned long long *>(T.p[k]) + (size_t)t * bm.m + j,
                          (unsigned long long)val);
            }
        }
    }
}


bool sq_accum_ready = false;

template <int NC>
cs_status sq_launch(SubqHandle &h, int rel, const uint32_t *keys, const int64_t *weights, uint64_t n, bool unit,
                    hipStream_t s)
{
    const SqRel &R = h.rel[rel];
    SqDesc D{};
    D.nt = (int32_t)R.targets.size();
    D.ns = (int32_t)R.sev.size();
    for (int c = 0, e = 0; c <= kSqMaxCols; ++c) {
        while (e < D.ns && R.sev[e].first < c) ++e;
        D.s_beg[c] = e;
    }
    SqTargets T{};
    for (int i = 0; i < D.nt; ++i) {
        D.col_mask[i] = R.col_mask[i];
        D.sign_mask[i] = R.sign_mask[i];
        T.p[i] = reinterpret_cast<uint64_t *>(h.counters + (size_t)R.targets[i] * h.d * h.m);
    }
    const BinMod bm = make_binmod(h.m);
    const int d = (int)h.d;
    if (weights && !unit) {
        const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 8192);
        hipLaunchKernelGGL(k_subq_atomic<NC>, dim3(grid), dim3(256), 0, s, keys, weights, n, R.coef_dev, R.cpr, D,
                           bm, d, T);
        CSK_HIP(hipGetLastError());
        return CS_OK;
    }
    if (!sq_accum_ready) {
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_subq_accum),
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)((2 * kSqR + 1024) * sizeof(uint32_t))));
        sq_accum_ready = true;
    }
    int n_cu = 256;
    CSK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h.device));
    const int ranges = (int)((h.m + kSqR - 1) / kSqR);
    const uint64_t chunk = h.chunk_blocks * kSqBlk;
    uint16_t *rec = static_cast<uint16_t *>(h.scratch);
    uint16_t *tab = rec + (size_t)D.nt * d * h.chunk_blocks * kSqCap;
    for (uint64_t b = 0; b < n; b += chunk) {
        const uint64_t len = std::min<uint64_t>(chunk, n - b);
        const uint64_t nblk = (len + kSqBlk - 1) / kSqBlk;
        const int groups0 = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)d, (uint64_t)n_cu * 4 / nblk));
        const int rpg = (d + groups0 - 1) / groups0;
        const int groups = (d + rpg - 1) / rpg;
        const uint32_t *kp = keys + b * NC;
        const int64_t *wp = weights ? weights + b : nullptr;
        if (wp)
            hipLaunchKernelGGL((k_subq_hash<NC, true>), dim3((unsigned)nblk, groups), dim3(kSqB), 0, s, kp, wp, len,
                               R.coef_dev, R.cpr, D, bm, d, ranges, rpg, nblk, rec, tab);
        else
            hipLaunchKernelGGL((k_subq_hash<NC, false>), dim3((unsigned)nblk, groups), dim3(kSqB), 0, s, kp, wp, len,
                               R.coef_dev, R.cpr, D, bm, d, ranges, rpg, nblk, rec, tab);
        CSK_HIP(hipGetLastError());
        const size_t lds = (2 * kSqR + nblk) * sizeof(uint32_t);
        hipLaunchKernelGGL(k_subq_accum, dim3(ranges, D.nt * d), dim3(kSqAB), lds, s, rec, tab, nblk, ranges, h.m,
                           d, T);
        CSK_HIP(hipGetLastError());
    }
    return CS_OK;
}

__global__ void k_subq_zero(int64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

void sq_free(SubqHandle &h)
{
    for (SqRel &r : h.rel)
        if (r.coef_dev) (void)hipFree(r.coef_dev);
    if (h.counters) (void)hipFree(h.counters);
    if (h.scratch) (void)hipFree(h.scratch);
    for (SqQuery &q : h.sub) release_work(q.view.work);
    release_work(h.est);
}

}  // namespace
}  // namespace csk

using namespace csk;

extern "C" {

cs_status cs_subq_create(const cs_graph *graph, const uint32_t *sub_joins, int32_t n_sub, uint32_t m, uint32_t d,
                         uint64_t seed, cs_subq **out)
{
    if (!out) return fail(CS_EINVAL, "null output handle");
    *out = nullptr;
    if (m < 2 || m > (1u << kMaxLog2M)) return fail(CS_EINVAL, "m must be in [2, 2^20]");
    if (d < 1 || d > (uint32_t)kMaxD) return fail(CS_EINVAL, "d must be in [1, 64]");
    if (n_sub < 1 || n_sub > kSqMaxSub || !sub_joins) return fail(CS_EINVAL, "need 1..4096 sub-queries");
    cs_subq *hs = new (std::nothrow) cs_subq();
    if (!hs) return fail(CS_ENOMEM, "host allocation failed");
    SubqHandle &h = hs->h;
    auto bail = [&](cs_status st) {
        sq_free(h);
        delete hs;
        return st;
    };
    cs_status st = analyze_graph(graph, &h.g);
    if (st != CS_OK) return bail(st);
    const GraphPlan &G = h.g;
    const int r = G.n_rel, E = G.n_edge, Q = G.n_comp;
    for (int k = 0; k < r; ++k)
        if ((int)G.omega[k].size() > kSqMaxCols) return bail(fail(CS_EINVAL, "sub-query sketches take relations of at most 4 attributes"));
    h.m = m;
    h.d = d;
    h.seed = seed;
    // hash functions: per repetition and component a shared sign polynomial and a bin
    // polynomial; then per repetition and join its own sign polynomial
    h.comp_sign.resize((size_t)d * Q * 4);
    h.bin.resize((size_t)d * Q * 2);
    h.edge_sign.resize((size_t)d * E * 4);
    SplitMix64 rng{seed};
    for (uint32_t t = 0; t < d; ++t)
        for (int q = 0; q < Q; ++q) {
            for (int i = 0; i < 4; ++i) h.comp_sign[((size_t)t * Q + q) * 4 + i] = rng.coef();
            for (int i = 0; i < 2; ++i) h.bin[((size_t)t * Q + q) * 2 + i] = rng.coef();
        }
    for (uint32_t t = 0; t < d; ++t)
        for (int e = 0; e < E; ++e)
            for (int i = 0; i < 4; ++i) h.edge_sign[((size_t)t * E + e) * 4 + i] = rng.coef();

    // sub-queries: their relations, the signature of each relation's sketch, the targets
    h.rel.resize(r);
    for (int k = 0; k < r; ++k) h.rel[k].a = (int)G.omega[k].size();
    std::map<std::vector<int>, int> tkey;  // (relation, per column: column, #ids, ids...) -> target
    std::vector<std::vector<int>> q_target(n_sub);
    h.sub.resize(n_sub);
    for (int qi = 0; qi < n_sub; ++qi) {
        const uint32_t mask = sub_joins[qi];
        if (mask == 0 || (E < 32 && (mask >> E) != 0)) return bail(fail(CS_EINVAL, "sub-query joins out of range"));
        SqQuery &S = h.sub[qi];
        S.mask = mask;
        std::vector<char> in_rel(r, 0);
        std::vector<int> joins_in_comp(Q, 0);
        std::vector<std::vector<int>> gq(G.n_attr);  // joins of the sub-query at each attribute
        int ne = 0;
        for (int e = 0; e < E; ++e) {
            if (!((mask >> e) & 1u)) continue;
            ++ne;
            const int u = G.edges[2 * e], v = G.edges[2 * e + 1];
            in_rel[G.attr_rel[u]] = in_rel[G.attr_rel[v]] = 1;
            joins_in_comp[G.psi[u]]++;
            gq[u].push_back(e);
            gq[v].push_back(e);
        }
        for (int k = 0; k < r; ++k)
            if (in_rel[k]) S.rels.push_back(k);
        // the base query is a tree of relations, so a set of its joins is connected
        // exactly when it touches one relation more than it has joins
        if ((int)S.rels.size() != ne + 1) return bail(fail(CS_EINVAL, "sub-query joins are not connected"));
        // the induced query, renumbered in ascending base order
        std::vector<int> rel_local(r, -1), attr_local(G.n_attr, -1);
        for (size_t i = 0; i < S.rels.size(); ++i) rel_local[S.rels[i]] = (int)i;
        std::vector<int32_t> attr_rel, edges;
        for (int u = 0; u < G.n_attr; ++u)
            if (!gq[u].empty()) {
                attr_local[u] = (int)attr_rel.size();
                attr_rel.push_back(rel_local[G.attr_rel[u]]);
            }
        for (int e = 0; e < E; ++e)
            if ((mask >> e) & 1u) {
                edges.push_back(attr_local[G.edges[2 * e]]);
                edges.push_back(attr_local[G.edges[2 * e + 1]]);
            }
        cs_graph lg{(int32_t)S.rels.size(), (int32_t)attr_rel.size(), attr_rel.data(), (int32_t)(edges.size() / 2),
                    edges.data()};
        Handle &V = S.view;
        st = analyze_graph(&lg, &V.g);
        if (st != CS_OK) return bail(st);
        V.m = m;
        V.log2m = 31 - __builtin_clz(m);
        V.pow2 = (m & (m - 1)) == 0;
        if (!V.pow2 && V.g.plan == CS_PLAN_SPECTRAL) V.g.plan = CS_PLAN_GENERAL;
        V.d = d;
        V.seed = seed;
        for (int k : S.rels) {
            std::vector<int> key{k};
            SqTarget tg;
            tg.rel = k;
            for (int c = 0; c < (int)G.omega[k].size(); ++c) {
                const int u = G.omega[k][c];
                if (gq[u].empty()) continue;
                std::vector<int> ids;
                if (joins_in_comp[G.psi[u]] == 1) {
                    ids.push_back(G.psi[u]);
                } else {
                    std::vector<int> es = gq[u];
                    std::sort(es.begin(), es.end());
                    for (int e : es) ids.push_back(Q + e);
                }
                key.push_back(c);
                key.push_back((int)ids.size());
                key.insert(key.end(), ids.begin(), ids.end());
                tg.cols.push_back({c, ids});
            }
            auto it = tkey.find(key);
            int id;
            if (it == tkey.end()) {
                id = (int)h.targets.size();
                tkey.emplace(key, id);
                h.targets.push_back(tg);
                h.rel[k].targets.push_back(id);
            } else {
                id = it->second;
            }
            q_target[qi].push_back(id);
        }
    }
    // per relation: its sign evaluations, target masks and coefficient table
    std::vector<std::vector<uint64_t>> tabs(r);
    for (int k = 0; k < r; ++k) {
        SqRel &R = h.rel[k];
        if ((int)R.targets.size() > kSqMaxTargets)
            return bail(fail(CS_EINVAL, "more than 16 distinct sketches of one relation"));
        for (int id : R.targets)
            for (auto &cs : h.targets[id].cols)
                for (int sid : cs.second) R.sev.push_back({cs.first, sid});
        std::sort(R.sev.begin(), R.sev.end());
        R.sev.erase(std::unique(R.sev.begin(), R.sev.end()), R.sev.end());
        if ((int)R.sev.size() > kSqMaxSign)
            return bail(fail(CS_EINVAL, "more than 16 distinct sign hashes on one relation"));
        for (int id : R.targets) {
            uint32_t cm = 0, sm = 0;
            for (auto &cs : h.targets[id].cols) {
                cm |= 1u << cs.first;
                for (int sid : cs.second) {
                    const int e = (int)(std::lower_bound(R.sev.begin(), R.sev.end(), std::make_pair(cs.first, sid)) -
                                        R.sev.begin());
                    sm |= 1u << e;
                }
            }
            R.col_mask.push_back(cm);
            R.sign_mask.push_back(sm);
        }
        if (R.targets.empty()) continue;
        R.cpr = 2 * R.a + 4 * (int)R.sev.size();
        std::vector<uint64_t> tab((size_t)d * R.cpr);
        for (uint32_t t = 0; t < d; ++t) {
            uint64_t *o = tab.data() + (size_t)t * R.cpr;
            for (int c = 0; c < R.a; ++c) {
                const int q = G.psi[G.omega[k][c]];
                o[2 * c] = h.bin[((size_t)t * Q + q) * 2];
                o[2 * c + 1] = h.bin[((size_t)t * Q + q) * 2 + 1];
            }
            for (size_t e = 0; e < R.sev.size(); ++e) {
                const int sid = R.sev[e].second;
                const uint64_t *src = sid < Q ? &h.comp_sign[((size_t)t * Q + sid) * 4]
                                              : &h.edge_sign[((size_t)t * E + (sid - Q)) * 4];
                for (int i = 0; i < 4; ++i) o[2 * R.a + 4 * e + i] = src[i];
            }
        }
        tabs[k] = std::move(tab);
    }
    // the plan is complete and valid (checked on the host): from here on the device
    if (hipGetDevice(&h.device) != hipSuccess) return bail(fail(CS_EDEVICE, "no HIP device"));
    for (SqQuery &S : h.sub) S.view.device = h.device;
    for (int k = 0; k < r; ++k) {
        SqRel &R = h.rel[k];
        if (tabs[k].empty()) continue;
        if (hipMalloc(&R.coef_dev, tabs[k].size() * sizeof(uint64_t)) != hipSuccess)
            return bail(fail(CS_ENOMEM, "sub-query coefficients"));
        if (hipMemcpy(R.coef_dev, tabs[k].data(), tabs[k].size() * sizeof(uint64_t), hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(fail(CS_EDEVICE, "sub-query coefficient upload"));
    }
    // counters and the pass-1 scratch of one chunk
    const size_t nt = h.targets.size();
    const size_t cbytes = nt * d * (size_t)m * sizeof(int64_t);
    if (hipMalloc(&h.counters, cbytes) != hipSuccess) return bail(fail(CS_ENOMEM, "sub-query counters"));
    if (hipMemset(h.counters, 0, cbytes) != hipSuccess) return bail(fail(CS_EDEVICE, "sub-query counter init"));
    size_t nt_max = 1;
    for (const SqRel &R : h.rel) nt_max = std::max(nt_max, R.targets.size());
    const int ranges = (int)((m + kSqR - 1) / kSqR);
    const size_t per_block = nt_max * d * ((size_t)kSqCap + ranges + 1) * sizeof(uint16_t);
    h.chunk_blocks = std::max<size_t>(1, std::min<size_t>(1024, kSqScratchBudget / per_block));
    h.scratch_bytes = h.chunk_blocks * per_block + 256;
    if (hipMalloc(&h.scratch, h.scratch_bytes) != hipSuccess) return bail(fail(CS_ENOMEM, "sub-query scratch"));
    for (int qi = 0; qi < n_sub; ++qi) {
        SqQuery &S = h.sub[qi];
        for (int id : q_target[qi]) S.view.rel_ptr.push_back(h.counters + (size_t)id * d * m);
    }
    if (hipStreamSynchronize(nullptr) != hipSuccess) return bail(fail(CS_EDEVICE, "sub-query initialisation"));
    *out = hs;
    return CS_OK;
}

cs_status cs_subq_destroy(cs_subq *hs)
{
    if (!hs) return CS_OK;
    (void)hipDeviceSynchronize();
    sq_free(hs->h);
    delete hs;
    return CS_OK;
}

cs_status cs_subq_update(cs_subq *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                         int32_t flags, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    SubqHandle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n == 0 || h.rel[rel].targets.empty()) return CS_OK;
    if (!keys) return fail(CS_EINVAL, "null keys");
    const int a = h.rel[rel].a;
    if (n > (~0ull) / 64) return fail(CS_EINVAL, "too many tuples");
    cs_status chk = check_device_array(keys, n * a * sizeof(uint32_t), h.device, "keys");
    if (chk == CS_OK && weights) chk = check_device_array(weights, n * sizeof(int64_t), h.device, "weights");
    if (chk != CS_OK) return chk;
    const bool unit = weights == nullptr || (flags & CS_UPDATE_UNIT_WEIGHTS) != 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (a) {
        case 1: return sq_launch<1>(h, rel, keys, weights, n, unit, s);
        case 2: return sq_launch<2>(h, rel, keys, weights, n, unit, s);
        case 3: return sq_launch<3>(h, rel, keys, weights, n, unit, s);
        default: return sq_launch<4>(h, rel, keys, weights, n, unit, s);
    }
}

cs_status cs_subq_reset(cs_subq *hs, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    SubqHandle &h = hs->h;
    const size_t n = h.targets.size() * h.d * (size_t)h.m;
    hipLaunchKernelGGL(k_subq_zero, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h.counters, n);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

cs_status cs_subq_estimate(cs_subq *hs, int32_t q, void *stream, cs_estimate_t *out, const cs_reps_t *reps)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    SubqHandle &h = hs->h;
    if (q < 0 || q >= (int)h.sub.size()) return fail(CS_EINVAL, "sub-query out of range");
    return estimate_run(h.sub[q].view, static_cast<hipStream_t>(stream), out, reps);
}

cs_status cs_subq_estimate_all(cs_subq *hs, void *stream, cs_estimate_t *outs)
{
    if (!hs || !outs) return fail(CS_EINVAL, "null argument");
    SubqHandle &h = hs->h;
    std::vector<Handle *> v(h.sub.size());
    for (size_t i = 0; i < h.sub.size(); ++i) v[i] = &h.sub[i].view;
    return estimate_batch(v.data(), (int)v.size(), static_cast<hipStream_t>(stream), outs, nullptr, h.est);
}

cs_status cs_subq_layout(const cs_subq *hs, int32_t *n_targets, int32_t *target_of)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    const SubqHandle &h = hs->h;
    if (n_targets) *n_targets = (int32_t)h.targets.size();
    if (target_of) {
        const int r = h.g.n_rel;
        for (size_t qi = 0; qi < h.sub.size(); ++qi) {
            int32_t *row = target_of + qi * r;
            for (int k = 0; k < r; ++k) row[k] = -1;
            const SqQuery &S = h.sub[qi];
            for (size_t i = 0; i < S.rels.size(); ++i)
                row[S.rels[i]] = (int32_t)((S.view.rel_ptr[i] - h.counters) / ((size_t)h.d * h.m));
        }
    }
    return CS_OK;
}

cs_status cs_subq_read(const cs_subq *hs, int32_t target, int64_t *host_out)
{
    if (!hs || !host_out) return fail(CS_EINVAL, "null argument");
    const SubqHandle &h = hs->h;
    if (target < 0 || target >= (int32_t)h.targets.size()) return fail(CS_EINVAL, "target out of range");
    CSK_HIP(hipDeviceSynchronize());
    CSK_HIP(hipMemcpy(host_out, h.counters + (size_t)target * h.d * h.m, (size_t)h.d * h.m * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    return CS_OK;
}

cs_status cs_subq_coefficients(const cs_subq *hs, uint64_t *comp_sign, uint64_t *bin, uint64_t *join_sign)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    const SubqHandle &h = hs->h;
    if (comp_sign) std::memcpy(comp_sign, h.comp_sign.data(), h.comp_sign.size() * sizeof(uint64_t));
    if (bin) std::memcpy(bin, h.bin.data(), h.bin.size() * sizeof(uint64_t));
    if (join_sign) std::memcpy(join_sign, h.edge_sign.data(), h.edge_sign.size() * sizeof(uint64_t));
    return CS_OK;
}

}  // extern "C"
