// The sketch handle: graph plan, coefficients, counters and estimate work buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "csk_internal.h"
#include "csk_transform.h"

namespace csk {

// Host-side analysis of a join query (Sec. 2.6, Table 1).
struct GraphPlan {
    int32_t n_rel = 0, n_attr = 0, n_edge = 0, n_comp = 0;
    std::vector<int32_t> attr_rel;                 // [n_attr]
    std::vector<int32_t> edges;                    // [n_edge][2]
    std::vector<int32_t> psi;                      // component of each attribute
    std::vector<std::vector<int32_t>> omega;       // attributes of each relation, ascending
    std::vector<std::vector<int32_t>> gamma;       // attributes joined with u, ascending
    std::vector<std::vector<int32_t>> gamma_edge;  // join index of (u, gamma[u][i])
    std::vector<int32_t> comp_size;                // attributes per component
    int32_t plan = 0;                              // cs_plan_kind
    uint32_t conj_mask = 0;                        // spectral plan: relations taken conjugated
    std::vector<Op> ops;                           // general plan: Alg. 3 as register ops
    int32_t n_regs = 0;
    int32_t result_reg = -1;
    std::vector<RelPlan> rel;                      // update plans
};

cs_status analyze_graph(const cs_graph *g, GraphPlan *out);

// Estimate work buffers, grown on demand and kept by the handle.
struct EstimateWork {
    void *buf = nullptr;        // one device allocation carved into the pieces below
    size_t bytes = 0;
    void *mod = nullptr;        // device workspace of the modular (exact) step
    size_t mod_bytes = 0;
    void *host = nullptr;       // pinned host staging: tables up, results down
    size_t host_bytes = 0;
    int spec_k = -1;            // primes the last estimate's repetitions needed (-1: no estimate yet)
    hipEvent_t ev_upload = nullptr;  // an asynchronous estimate's table upload
    bool upload_pending = false;     // host staging still being read by that upload
    hipStream_t side = nullptr;      // the speculative modular chain's stream (default priority)
    hipEvent_t ev_fork = nullptr;    // its start behind the table upload
    hipEvent_t ev_join = nullptr;    // its end, waited on before the finalize
};
// Frees every buffer of a workspace (the device must be idle for it).
void release_work(EstimateWork &w);

struct Handle {
    int device = 0;
    uint32_t m = 0;
    int32_t log2m = 0;
    bool pow2 = true;
    uint32_t d = 0;
    uint64_t seed = 0;
    GraphPlan g;
    std::vector<uint64_t> sign_coef;   // [d][E][4]
    std::vector<uint64_t> bin_coef;    // [d][Q][2]
    int64_t *counters = nullptr;       // [r][d][m]
    // when set, relation k's [d][m] counters live at rel_ptr[k] instead (handles that
    // only estimate, over sketches owned elsewhere)
    std::vector<int64_t *> rel_ptr;
    uint64_t *coef_dev = nullptr;      // per relation: [d][coef_per_rep], concatenated
    std::vector<size_t> coef_off;      // offset of relation k's table in coef_dev
    EstimateWork work;
    bool own_scratch = false;          // the handle keeps its own update scratch (grown on demand)
    void *scratch = nullptr;           // partial sums of the LDS-segmented update, partition records
    size_t scratch_bytes = 0;
    void *filter_scratch = nullptr;    // filtered 16-bit path: partial sums and a round of kept keys
    size_t filter_scratch_bytes = 0;   //   (allocated by the first filtered update that needs it)
    void *result_host = nullptr;       // pinned host staging for results
    // two device words: [0] the kept tuples of a filtered update that asked for the
    // count, [1] the per-round count of the filtered 16-bit path (zero between updates)
    // two words of the filtered update (kept count, per-round count), followed by the
    // partition strategy's hot-key hints PartHints[r] (one allocation)
    unsigned long long *kept_dev = nullptr;
};

// Relation k's counters [d][m].
inline int64_t *rel_counters(const Handle &h, int k)
{
    return h.rel_ptr.empty() ? h.counters + (size_t)k * h.d * h.m : h.rel_ptr[k];
}

cs_status estimate_run(Handle &h, hipStream_t s, cs_estimate_t *out, const cs_reps_t *reps);
cs_status estimate_run_async(Handle &h, hipStream_t s, cs_estimate_t *out);
}  // namespace csk
struct cs_sketch;
namespace csk {
// Handle creation; without scratch the handle serves batched and served updates only.
cs_status create_handle(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, bool with_scratch,
                        cs_sketch **out);
// Grows the handle's own update scratch to what an update of n tuples can use (waiting
// for `s` before freeing the old buffer; calls on one handle are ordered by their
// stream); handles without their own scratch are left alone.
cs_status ensure_scratch(cs_sketch *hs, uint64_t n, const int64_t *weights, int32_t flags, hipStream_t s);
// Checks the arguments of an update of relation rel and fills the launcher's arguments
// (keys, weights, coefficients, counters, the handle's scratch, flags).
cs_status update_args(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                      int32_t flags, UpdateArgs *out);
// Estimates of nq queries at once (one FFT launch per sketch length, one product-reduce
// launch per length, one finalize launch); reps_out may be null or hold nq entries.
cs_status estimate_batch(Handle *const *hs, int nq, hipStream_t s, cs_estimate_t *outs, const cs_reps_t *reps_out,
                         EstimateWork &ws, cs_estimate_t *async_out = nullptr);

}  // namespace csk

// The opaque handle of the C ABI.
struct cs_sketch {
    csk::Handle h;
};
