// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/csketch.h"

namespace csk {

constexpr int kMaxRel = 16;
constexpr int kMaxAttr = 32;
constexpr int kMaxCols = 8;          // attributes per relation
constexpr int kMaxEdgesPerAttr = 8;  // joins per attribute
constexpr int kMaxD = 64;
constexpr int kMaxLog2M = 20;
constexpr int kMaxLog2N = kMaxLog2M + 1;  // longest transform: a zero-padded correlation for m not a power of two
constexpr int kMaxPrimes = 12;       // modular path: up to ~370-bit results
constexpr uint64_t kP61 = (1ull << 61) - 1;

// SplitMix64 (Steele, Lea & Flood 2014).
// Coefficients are its outputs shifted right by 3, redrawn when equal to p.
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint64_t coef()
    {
        for (;;) {
            const uint64_t c = next() >> 3;
            if (c != kP61) return c;
        }
    }
};


// ------------------------------------------------------------------ errors

void set_error(const std::string &msg);
cs_status fail(cs_status st, const std::string &msg);
// CS_OK when the bytes [p, p + bytes) start and end in memory the given device's kernels
// can read (its own device memory, or pinned / managed host memory); otherwise
// CS_EINVAL naming `what`.  A null p with bytes == 0 passes.  Kernels reading pageable
// host memory would fault the GPU, so every entry point that hands caller arrays to a
// kernel checks them first.
cs_status check_device_array(const void *p, size_t bytes, int device, const char *what);
#define CSK_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess)                                                          \
            return ::csk::fail(CS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Record an optional timing event on stream s (inside functions returning cs_status).
#define CSK_MARK(ev, s)                                \
    do {                                               \
        if (ev) CSK_HIP(hipEventRecord((ev), (s)));    \
    } while (0)

// ------------------------------------------------------------------ plans

// Per-relation hashing plan: key column c carries attribute omega[c]; its bin hash is
// the component's, and its sign is the product over the joins at that attribute.
// The coefficients of one repetition are laid out for the update kernel as, for each
// column in order: b0, b1, then a0..a3 of each join at the column.
struct RelPlan {
    int32_t n_cols;
    int32_t coef_per_rep;             // u64 coefficients per repetition
    int32_t n_edges[kMaxCols];        // joins per column
};

// Modular op list (Alg. 3 in modular arithmetic) for general queries.
enum OpCode : int32_t { OP_LOAD = 0, OP_ONES = 1, OP_HAD = 2, OP_CORR = 3 };
struct Op {
    int32_t code;
    int32_t dst;   // register
    int32_t src;   // register (HAD: dst *= src; CORR: dst = src star dst) or relation (LOAD)
};

struct Handle;  // defined in csk_api.cpp

// ------------------------------------------------------------------ modular primes

struct PrimeInfo {
    uint32_t p;
    uint32_t pinv_neg;   // -p^{-1} mod 2^32
    uint32_t r2;         // 2^64 mod p   (R^2, R = 2^32)
    uint32_t r3;         // 2^96 mod p   (R^3)
    uint32_t neg2_64;    // (-2^64 * R) mod p: Montgomery form of -2^64
    uint32_t g;          // generator of the multiplicative group
};
// NTT primes p < 2^31 with 2^kMaxLog2N | p - 1, largest first (host table).
const std::vector<PrimeInfo> &ntt_primes();

// ------------------------------------------------------------------ device tables

// Twiddles exp(-2 pi i k / 2^L) for k < 2^L, fp64 complex interleaved, cached per
// device and L.  Computed on the host in long double.
const double *twiddles_f64(int device, int log2m, hipStream_t s, cs_status *st);
// Montgomery-form powers of a primitive 2^L-th root of unity mod prime i (forward and
// inverse tables, each 2^L entries), cached per device, L and prime.
const uint32_t *roots_mod(int device, int log2m, int prime, bool inverse, hipStream_t s,
                          cs_status *st);

// ------------------------------------------------------------------ launchers

// Conjunction of range predicates lo <= attrs[i][col] <= hi (ingestion filters).
struct FilterSpec {
    int32_t n;
    int32_t col[CS_MAX_PREDICATES];
    uint32_t lo[CS_MAX_PREDICATES], hi[CS_MAX_PREDICATES];
};

struct PartHints;
struct UpdateArgs {
    const uint32_t *keys;
    const int64_t *weights;
    uint64_t n;
    const uint64_t *coef;   // [d][coef_per_rep]
    uint64_t *sketch;       // [d][m]
    uint32_t m;
    int32_t d;
    RelPlan plan;
    void *scratch;          // partial-sum buffer of the LDS-segmented strategy (may be null)
    size_t scratch_bytes;
    bool unit_weights;      // caller guarantees every weight is +1 or -1
    bool compact = true;    // segmented strategy: compacting kernel for bucket-range segments
    bool counters16 = true; // segmented strategy: 16-bit LDS counters when they hold a repetition
    // hashes whose flag (CoefE1::bin_neg_fast) reaches this take the full reduction; the
    // exact bound is 0xFFFFFFFF, a test lowers it to send half of them that way
    uint32_t canon_thresh = 0xFFFFFFFFu;
    hipEvent_t ev_start = nullptr;  // recorded just before / after the hashing kernel(s)
    hipEvent_t ev_stop = nullptr;
    // ingestion filter (cs_update_filtered): only tuples whose attribute columns
    // attrs [n][n_attrs] pass every predicate are sketched; kept, when set, is a device
    // counter the kernels add the number of kept tuples to
    const FilterSpec *filter = nullptr;
    const uint32_t *attrs = nullptr;
    int32_t n_attrs = 0;
    unsigned long long *kept = nullptr;
    // a device word that is zero between filtered updates (the handle's), used by the
    // filtered 16-bit path for its per-round count of kept tuples
    unsigned long long *filter_count = nullptr;
    // the relation's hot-tuple hints (partition strategy; may be null)
    PartHints *hints = nullptr;
};
struct SegGeom {
    uint32_t R;        // counter cells per segment
    int32_t segments;  // segments covering [d][m]
    int32_t chunks;    // tuple chunks (partial buffers)
};
// n: tuples of the update (chunks shrink for small inputs); the default sizes buffers.
SegGeom seg_geometry(uint32_t m, int32_t d, bool narrow, size_t scratch_bytes, uint64_t n = ~0ull);
SegGeom seg16_geometry(uint32_t m, int32_t d, size_t scratch_bytes, uint64_t n = ~0ull);
constexpr int kMaxPartRanges = 64;           // bucket ranges of 2^14 per repetition (m <= 2^20)
constexpr uint64_t kPartMaxChunk = 1ull << 23;  // tuples per pass pair (2048 blocks: pass 2 keeps a run word per block in LDS)
// One block's hot tuples for the partition strategy (see k_part_hash): up to eight
// tuples (keys; column 1 unused for one-column relations) and their Delta sums.
constexpr int kPartHot = 8;
struct PartHot {
    uint32_t key[kPartHot][2];
    int32_t sum[kPartHot];
};
// A relation's most frequent hot tuples over the blocks of its last partition update
// (n of them, hottest first), offered to the next update of that relation as election
// candidates before its own sampled tuples.  Any content gives the same counters: a
// candidate is elected only on its count in the block's sample.
struct PartHints {
    uint32_t n;
    uint32_t key[kPartHot][2];
};
struct PartGeom {
    int32_t ranges;          // bucket ranges of 2^14 per repetition (the last may be partial)
    uint64_t chunk;          // tuples per pass pair (a multiple of the 1024-tuple segment)
    uint64_t nseg;           // segments per chunk
    size_t tab_offset;       // range starts after the records in the scratch buffer
    size_t hot_offset;       // hot-tuple list after the range starts
    int32_t groups;          // pass-1 repetition groups
    int32_t reps_per_group;
};
PartGeom part_geometry(uint32_t m, int32_t d, size_t scratch_bytes);
size_t seg_scratch_bytes(uint32_t m, int32_t d);
// What the update strategies can use for one call of n tuples (unit: Deltas +-1), no
// more than seg_scratch_bytes.
size_t update_scratch_bytes(uint32_t m, int32_t d, uint64_t n, bool unit);
// Scratch of the filtered 16-bit path (2^15 < m <= 2^16; 0 elsewhere): a handle
// allocates it on its first filtered update of that shape.
size_t filter_scratch_bytes(uint32_t m, int32_t d);
cs_status launch_update(const UpdateArgs &a, int strategy, int grid_blocks, hipStream_t s);
// Sets a device word to zero with a one-thread kernel on s (no memset node, so it can be
// captured into a graph).
cs_status zero_device_u64(unsigned long long *p, hipStream_t s);
// Tuned (strategy, grid, flags) for this update's class on `device`, if one was tuned.
bool tune_lookup(const UpdateArgs &a, int device, int *strategy, int *grid, int *flags);
// Batched update tasks: kind (0 global atomics, 1 LDS segment) and log2 of the tuples per
// task tuned for the class (device, m, d, key columns, one-join columns, unit weights,
// floor(log2 n)).
bool tune_lookup_batch(int device, uint32_t m, int d, int n_cols, int e1, int unit, uint64_t n, int *kind,
                       int *chunk_log2);
void tune_store_batch(int device, uint32_t m, int d, int n_cols, int e1, int unit, uint64_t n, int kind,
                      int chunk_log2, float ms);
// Row length 2^S tuned for two-pass transforms of length 2^log2m (0: none tuned).
int tune_split(int device, int log2m);
void tune_store_split(int device, int log2m, int S, float ms);
// Whether 2^S is a usable row length for a two-pass transform of length 2^log2m: tiles of
// 2^10..2^12 elements, columns no longer than rows.
inline bool split_ok(int log2m, int S) { return S >= 10 && S <= 12 && 2 * S >= log2m && S < log2m; }
int auto_update_strategy(uint32_t m, int32_t d, uint64_t n, int n_cols, bool unit, bool has_scratch,
                         bool e1_pow2);

}  // namespace csk
