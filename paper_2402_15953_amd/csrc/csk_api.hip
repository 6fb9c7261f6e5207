// C ABI entry points: handle lifecycle, join-graph analysis, hash coefficient sampling
// (Alg. 1: SampleSignHashes, SampleBinHashes), update and estimate dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "csk_handle.h"
#include "csk_internal.h"

namespace csk {

namespace {
thread_local std::string g_err;

// Zeroes n int64 (the counter block is 256-byte aligned): 16-byte stores, then the tail.
__global__ void k_fill_zero(int64_t *p, size_t n)
{
    const size_t n2 = n / 2;
    longlong2 *q = reinterpret_cast<longlong2 *>(p);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (size_t)gridDim.x * blockDim.x)
        q[i] = make_longlong2(0, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) p[n - 1] = 0;
}

__global__ void k_add_i64(int64_t *dst, const int64_t *src, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (int64_t)((uint64_t)dst[i] + (uint64_t)src[i]);
}


}  // namespace

void set_error(const std::string &msg) { g_err = msg; }

cs_status fail(cs_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

cs_status check_device_array(const void *p, size_t bytes, int device, const char *what)
{
    if (bytes == 0) return CS_OK;
    if (!p) return fail(CS_EINVAL, std::string("null ") + what);
    const char *c = static_cast<const char *>(p);
    for (const char *q : {c, c + bytes - 1}) {
        hipPointerAttribute_t attr{};
        if (hipPointerGetAttributes(&attr, q) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CS_EINVAL, std::string(what) + " is not device or pinned host memory");
        }
        if (attr.type == hipMemoryTypeDevice) {
            if (attr.device != device) return fail(CS_EINVAL, std::string(what) + " is on another device");
        } else if (attr.type != hipMemoryTypeHost && attr.type != hipMemoryTypeManaged) {
            return fail(CS_EINVAL, std::string(what) + " is not device or pinned host memory");
        }
    }
    return CS_OK;
}

// Graph analysis (Sec. 2.6, Table 1): Omega, Gamma, Psi; validity; estimate plan.
cs_status analyze_graph(const cs_graph *g, GraphPlan *out)
{
    if (!g || !g->attr_rel || (g->n_edge > 0 && !g->edges)) return fail(CS_EINVAL, "null graph");
    const int r = g->n_rel, w = g->n_attr, ne = g->n_edge;
    if (r < 2 || r > kMaxRel) return fail(CS_EGRAPH, "need 2..16 relations");
    if (w < 2 || w > kMaxAttr) return fail(CS_EGRAPH, "need 2..32 attributes");
    GraphPlan P;
    P.n_rel = r;
    P.n_attr = w;
    P.n_edge = ne;
    P.attr_rel.assign(g->attr_rel, g->attr_rel + w);
    P.edges.assign(g->edges, g->edges + 2 * ne);
    for (int u = 0; u < w; ++u)
        if (P.attr_rel[u] < 0 || P.attr_rel[u] >= r) return fail(CS_EGRAPH, "attribute owner out of range");
    P.omega.assign(r, {});
    for (int u = 0; u < w; ++u) P.omega[P.attr_rel[u]].push_back(u);
    for (int k = 0; k < r; ++k) {
        if (P.omega[k].empty()) return fail(CS_EGRAPH, "relation without joined attribute");
        if ((int)P.omega[k].size() > kMaxCols) return fail(CS_EGRAPH, "too many attributes in a relation");
    }
    P.gamma.assign(w, {});
    std::vector<std::vector<std::pair<int, int>>> nb(w);
    for (int e = 0; e < ne; ++e) {
        const int u = P.edges[2 * e], v = P.edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= w || v >= w || u == v) return fail(CS_EGRAPH, "bad join endpoints");
        if (P.attr_rel[u] == P.attr_rel[v]) return fail(CS_EGRAPH, "join inside one relation");
        for (auto &pv : nb[u])
            if (pv.first == v) return fail(CS_EGRAPH, "duplicate join");
        nb[u].push_back({v, e});
        nb[v].push_back({u, e});
    }
    P.gamma_edge.assign(w, {});
    for (int u = 0; u < w; ++u) {
        if (nb[u].empty()) return fail(CS_EGRAPH, "attribute not joined");
        if ((int)nb[u].size() > kMaxEdgesPerAttr) return fail(CS_EGRAPH, "too many joins at an attribute");
        std::sort(nb[u].begin(), nb[u].end());
        for (auto &pv : nb[u]) {
            P.gamma[u].push_back(pv.first);
            P.gamma_edge[u].push_back(pv.second);
        }
    }
    if (ne != r - 1) return fail(CS_EGRAPH, "the relations and joins must form a tree (n_edge = n_rel - 1)");
    std::vector<int> par(r);
    for (int k = 0; k < r; ++k) par[k] = k;
    std::function<int(int)> find = [&](int x) { return par[x] == x ? x : par[x] = find(par[x]); };
    for (int e = 0; e < ne; ++e) {
        const int a = find(P.attr_rel[P.edges[2 * e]]), b = find(P.attr_rel[P.edges[2 * e + 1]]);
        if (a == b) return fail(CS_EGRAPH, "cyclic query");
        par[a] = b;
    }
    for (int k = 1; k < r; ++k)
        if (find(k) != find(0)) return fail(CS_EGRAPH, "query not connected");
    // components numbered by smallest attribute id
    P.psi.assign(w, -1);
    for (int u = 0; u < w; ++u) {
        if (P.psi[u] >= 0) continue;
        const int q = P.n_comp++;
        std::vector<int> st{u};
        P.psi[u] = q;
        while (!st.empty()) {
            const int a = st.back();
            st.pop_back();
            for (int b : P.gamma[a])
                if (P.psi[b] < 0) {
                    P.psi[b] = q;
                    st.push_back(b);
                }
        }
    }
    P.comp_size.assign(P.n_comp, 0);
    for (int u = 0; u < w; ++u) P.comp_size[P.psi[u]]++;
    // update plans: per column, the component's bin coefficients then each join's signs
    P.rel.resize(r);
    for (int k = 0; k < r; ++k) {
        RelPlan &rp = P.rel[k];
        std::memset(&rp, 0, sizeof(rp));
        rp.n_cols = (int)P.omega[k].size();
        int cpr = 0;
        for (int c = 0; c < rp.n_cols; ++c) {
            const int u = P.omega[k][c];
            rp.n_edges[c] = (int)P.gamma[u].size();
            cpr += 2 + 4 * rp.n_edges[c];
        }
        rp.coef_per_rep = cpr;
    }
    // estimate plan
    bool pairwise = true;
    for (int q = 0; q < P.n_comp; ++q)
        if (P.comp_size[q] != 2) pairwise = false;
    if (r == 2) {
        P.plan = CS_PLAN_DOT;
    } else if (pairwise) {
        P.plan = CS_PLAN_SPECTRAL;
        // relation-tree depth parity from relation 0
        std::vector<int> depth(r, -1);
        depth[0] = 0;
        std::vector<int> queue{0};
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            const int k = queue[qi];
            for (int u : P.omega[k])
                for (int v : P.gamma[u]) {
                    const int k2 = P.attr_rel[v];
                    if (depth[k2] < 0) {
                        depth[k2] = depth[k] + 1;
                        queue.push_back(k2);
                    }
                }
        }
        P.conj_mask = 0;
        for (int k = 0; k < r; ++k)
            if (depth[k] & 1) P.conj_mask |= 1u << k;
    } else {
        P.plan = CS_PLAN_GENERAL;
    }
    if (r > 2) {
        // Alg. 3 (CombineSketches from root attribute 0) compiled to register ops: the
        // general plan's program, and the spectral plan's when m is not a power of two.
        std::vector<int> free_regs;
        int n_regs = 0;
        auto alloc = [&]() {
            if (!free_regs.empty()) {
                const int x = free_regs.back();
                free_regs.pop_back();
                return x;
            }
            return n_regs++;
        };
        std::vector<char> visited(w, 0);
        std::function<int(int)> combine = [&](int u) -> int {
            const int k = P.attr_rel[u];
            const int x = alloc();
            P.ops.push_back({OP_LOAD, x, k});
            visited[u] = 1;
            for (int u2 : P.omega[k]) {
                if (u2 == u) continue;
                visited[u2] = 1;
                const int a = alloc();
                P.ops.push_back({OP_ONES, a, 0});
                for (int v : P.gamma[u2]) {
                    const int y = combine(v);
                    P.ops.push_back({OP_HAD, a, y});
                    free_regs.push_back(y);
                }
                P.ops.push_back({OP_CORR, x, a});
                free_regs.push_back(a);
            }
            for (int v : P.gamma[u]) {
                if (visited[v]) continue;
                const int y = combine(v);
                P.ops.push_back({OP_HAD, x, y});
                free_regs.push_back(y);
            }
            return x;
        };
        P.result_reg = combine(0);
        P.n_regs = n_regs;
    }
    *out = std::move(P);
    return CS_OK;
}

}  // namespace csk

using namespace csk;


extern "C" {

const char *cs_last_error(void) { return g_err.c_str(); }

uint64_t cs_sketch_bytes(const cs_graph *graph, uint32_t m, uint32_t d)
{
    if (!graph || graph->n_rel <= 0 || m == 0 || d == 0) return 0;
    return (uint64_t)graph->n_rel * d * m * 8ull;
}

cs_status cs_create(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, cs_sketch **out)
{
    return create_handle(graph, m, d, seed, true, out);
}

}  // extern "C"

namespace csk {

// Handle creation; without scratch the handle serves batched and served updates only
// (cs_update then uses the global-atomic strategy).
cs_status create_handle(const cs_graph *graph, uint32_t m, uint32_t d, uint64_t seed, bool with_scratch,
                        cs_sketch **out)
{
    if (!out) return fail(CS_EINVAL, "null output handle");
    *out = nullptr;
    if (m < 2 || m > (1u << kMaxLog2M)) return fail(CS_EINVAL, "m must be in [2, 2^20]");
    if (d < 1 || d > (uint32_t)kMaxD) return fail(CS_EINVAL, "d must be in [1, 64]");
    cs_sketch *hs = new (std::nothrow) cs_sketch();
    if (!hs) return fail(CS_ENOMEM, "host allocation failed");
    Handle &h = hs->h;
    cs_status st = analyze_graph(graph, &h.g);
    if (st != CS_OK) {
        delete hs;
        return st;
    }
    h.m = m;
    h.log2m = 31 - __builtin_clz(m);  // exact only when m is a power of two
    h.pow2 = (m & (m - 1)) == 0;
    // the frequency-domain plan needs power-of-two transforms; otherwise Alg. 3 runs as
    // its register program (time-domain correlations through zero-padded transforms)
    if (!h.pow2 && h.g.plan == CS_PLAN_SPECTRAL) h.g.plan = CS_PLAN_GENERAL;
    h.d = d;
    h.seed = seed;
    if (hipGetDevice(&h.device) != hipSuccess) {
        delete hs;
        return fail(CS_EDEVICE, "no HIP device");
    }
    // Alg. 1: sign hash per join (degree 3), bin hash per component (degree 1), per repetition
    const int E = h.g.n_edge, Q = h.g.n_comp;
    h.sign_coef.resize((size_t)d * E * 4);
    h.bin_coef.resize((size_t)d * Q * 2);
    SplitMix64 rng{seed};
    for (uint32_t t = 0; t < d; ++t) {
        for (int e = 0; e < E; ++e)
            for (int i = 0; i < 4; ++i) h.sign_coef[((size_t)t * E + e) * 4 + i] = rng.coef();
        for (int q = 0; q < Q; ++q)
            for (int i = 0; i < 2; ++i) h.bin_coef[((size_t)t * Q + q) * 2 + i] = rng.coef();
    }
    // per-relation coefficient tables in the update kernel's order
    std::vector<uint64_t> tab;
    h.coef_off.resize(h.g.n_rel);
    for (int k = 0; k < h.g.n_rel; ++k) {
        h.coef_off[k] = tab.size();
        for (uint32_t t = 0; t < d; ++t)
            for (int u : h.g.omega[k]) {
                const int q = h.g.psi[u];
                tab.push_back(h.bin_coef[((size_t)t * Q + q) * 2 + 0]);
                tab.push_back(h.bin_coef[((size_t)t * Q + q) * 2 + 1]);
                for (size_t i = 0; i < h.g.gamma[u].size(); ++i) {
                    const int e = h.g.gamma_edge[u][i];
                    for (int c = 0; c < 4; ++c) tab.push_back(h.sign_coef[((size_t)t * E + e) * 4 + c]);
                }
            }
    }
    const size_t n_ctr = (size_t)h.g.n_rel * d * m;
    if (hipMalloc(&h.counters, n_ctr * sizeof(int64_t)) != hipSuccess) {
        delete hs;
        return fail(CS_ENOMEM, "counter allocation failed");
    }
    if (hipMalloc(&h.coef_dev, tab.size() * sizeof(uint64_t)) != hipSuccess) {
        hipFree(h.counters);
        delete hs;
        return fail(CS_ENOMEM, "coefficient allocation failed");
    }
    // the update's scratch (partial sums, records) belongs to the handle: cs_update
    // orders itself against no other handle's updates; it is allocated by the first
    // update that needs it, sized for that update (and grown by a larger one)
    h.own_scratch = with_scratch;
    // one small allocation: the filter's two counters, then the relations' hot-key hints
    const size_t small_bytes = 2 * sizeof(unsigned long long) + (size_t)h.g.n_rel * sizeof(PartHints);
    if (hipMalloc(&h.kept_dev, small_bytes) != hipSuccess || hipMemset(h.kept_dev, 0, small_bytes) != hipSuccess ||
        hipMemcpy(h.coef_dev, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h.counters, 0, n_ctr * sizeof(int64_t)) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {  // the null stream only: other streams' work is not waited for
        hipFree(h.counters);
        hipFree(h.coef_dev);
        hipFree(h.scratch);
        hipFree(h.kept_dev);
        delete hs;
        return fail(CS_EDEVICE, "initialisation failed");
    }
    *out = hs;
    return CS_OK;
}

}  // namespace csk

extern "C" {

cs_status cs_destroy(cs_sketch *hs)
{
    if (!hs) return CS_OK;
    Handle &h = hs->h;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(h.device);
    hipDeviceSynchronize();
    if (h.counters) hipFree(h.counters);
    if (h.coef_dev) hipFree(h.coef_dev);
    release_work(h.work);
    if (h.scratch) hipFree(h.scratch);
    if (h.filter_scratch) hipFree(h.filter_scratch);
    if (h.kept_dev) hipFree(h.kept_dev);  // the hints share this allocation
    hipSetDevice(cur);
    delete hs;
    return CS_OK;
}

cs_status cs_get_info(const cs_sketch *hs, cs_info_t *out)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    const Handle &h = hs->h;
    out->n_rel = h.g.n_rel;
    out->n_attr = h.g.n_attr;
    out->n_edge = h.g.n_edge;
    out->n_comp = h.g.n_comp;
    out->m = h.m;
    out->d = h.d;
    out->plan = h.g.plan;
    out->device = h.device;
    out->counter_bytes = (uint64_t)h.g.n_rel * h.d * h.m * 8ull;
    out->workspace_bytes = h.work.bytes;
    return CS_OK;
}

cs_status cs_update_ex(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                       void *stream, int32_t strategy, int32_t grid_blocks, int32_t flags)
{
    return cs_update_timed(hs, rel, keys, weights, n, stream, strategy, grid_blocks, flags, nullptr, nullptr);
}

}  // extern "C"

namespace csk {

cs_status ensure_scratch(cs_sketch *hs, uint64_t n, const int64_t *weights, int32_t flags, hipStream_t s)
{
    Handle &h = hs->h;
    if (!h.own_scratch || n == 0) return CS_OK;
    const bool unit = weights == nullptr || (flags & CS_UPDATE_UNIT_WEIGHTS) != 0;
    const size_t need = update_scratch_bytes(h.m, (int32_t)h.d, n, unit);
    if (h.scratch_bytes >= need) return CS_OK;
    CSK_HIP(hipStreamSynchronize(s));
    if (h.scratch) (void)hipFree(h.scratch);
    h.scratch = nullptr;
    h.scratch_bytes = 0;
    if (hipMalloc(&h.scratch, need) != hipSuccess) {
        h.scratch = nullptr;
        return fail(CS_ENOMEM, "update scratch allocation failed");
    }
    h.scratch_bytes = need;
    return CS_OK;
}

cs_status update_args(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                      int32_t flags, UpdateArgs *out)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    Handle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n > 0 && !keys) return fail(CS_EINVAL, "null keys");
    if (n > 0) {
        cs_status chk = check_device_array(keys, n * h.g.rel[rel].n_cols * sizeof(uint32_t), h.device, "keys");
        if (chk == CS_OK && weights) chk = check_device_array(weights, n * sizeof(int64_t), h.device, "weights");
        if (chk != CS_OK) return chk;
    }
    UpdateArgs &a = *out;
    a.keys = keys;
    a.weights = weights;
    a.n = n;
    a.coef = h.coef_dev + h.coef_off[rel];
    a.sketch = reinterpret_cast<uint64_t *>(h.counters + (size_t)rel * h.d * h.m);
    a.m = h.m;
    a.d = (int32_t)h.d;
    a.plan = h.g.rel[rel];
    a.scratch = h.scratch;
    a.scratch_bytes = h.scratch_bytes;
    a.filter_count = h.kept_dev ? h.kept_dev + 1 : nullptr;
    a.hints = h.kept_dev ? reinterpret_cast<PartHints *>(h.kept_dev + 2) + rel : nullptr;
    a.unit_weights = (flags & CS_UPDATE_UNIT_WEIGHTS) != 0;
    a.compact = (flags & CS_UPDATE_NO_COMPACT) == 0;
    a.counters16 = (flags & CS_UPDATE_NO_COUNTERS16) == 0;
    if (flags & CS_UPDATE_TEST_FULL_REDUCTION) a.canon_thresh = 0xF0000000u;
    return CS_OK;
}

}  // namespace csk

extern "C" {

cs_status cs_update_timed(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                          void *stream, int32_t strategy, int32_t grid_blocks, int32_t flags, void *ev_start,
                          void *ev_stop)
{
    if (strategy < CS_UPDATE_AUTO || strategy > CS_UPDATE_PARTITION) return fail(CS_EINVAL, "bad strategy");
    UpdateArgs a;
    cs_status st = update_args(hs, rel, keys, weights, n, flags, &a);
    if (st != CS_OK || n == 0) return st;
    if ((st = ensure_scratch(hs, n, weights, flags, static_cast<hipStream_t>(stream))) != CS_OK) return st;
    a.scratch = hs->h.scratch;
    a.scratch_bytes = hs->h.scratch_bytes;
    a.ev_start = static_cast<hipEvent_t>(ev_start);
    a.ev_stop = static_cast<hipEvent_t>(ev_stop);
    return launch_update(a, strategy, grid_blocks, static_cast<hipStream_t>(stream));
}

cs_status cs_update_filtered(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                             const uint32_t *attrs, int32_t n_attrs, const cs_predicate *preds, int32_t n_preds,
                             int32_t flags, void *stream, uint64_t *n_kept)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    Handle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n_kept) *n_kept = 0;
    if (n == 0) return CS_OK;
    if (!keys) return fail(CS_EINVAL, "null keys");
    if (n_preds < 0 || n_preds > CS_MAX_PREDICATES) return fail(CS_EINVAL, "too many predicates");
    if (n_preds > 0 && (!preds || !attrs || n_attrs <= 0 || n_attrs > CS_MAX_PREDICATES))
        return fail(CS_EINVAL, "predicates need attribute columns");
    {
        cs_status chk = check_device_array(keys, n * h.g.rel[rel].n_cols * sizeof(uint32_t), h.device, "keys");
        if (chk == CS_OK && weights) chk = check_device_array(weights, n * sizeof(int64_t), h.device, "weights");
        if (chk == CS_OK && n_preds > 0)
            chk = check_device_array(attrs, n * (size_t)n_attrs * sizeof(uint32_t), h.device, "attribute columns");
        if (chk != CS_OK) return chk;
    }
    FilterSpec f{};
    f.n = n_preds;
    for (int i = 0; i < n_preds; ++i) {
        if (preds[i].column < 0 || preds[i].column >= n_attrs) return fail(CS_EINVAL, "predicate column out of range");
        f.col[i] = preds[i].column;
        f.lo[i] = preds[i].lo;
        f.hi[i] = preds[i].hi;
    }
    if (n_preds == 0) {  // nothing to filter
        if (n_kept) *n_kept = n;
        return cs_update_ex(hs, rel, keys, weights, n, stream, CS_UPDATE_AUTO, 0, flags);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    UpdateArgs a;
    cs_status st = update_args(hs, rel, keys, weights, n, flags, &a);
    if (st != CS_OK) return st;
    if ((st = ensure_scratch(hs, n, weights, flags, s)) != CS_OK) return st;
    a.scratch = h.scratch;
    a.scratch_bytes = h.scratch_bytes;
    a.filter = &f;
    a.attrs = attrs;
    a.n_attrs = n_attrs;
    const size_t fb = filter_scratch_bytes(h.m, (int32_t)h.d);
    if (fb > 0 && a.scratch) {
        // the 16-bit filtered path keeps a round of kept keys beside its partial sums:
        // allocated once per handle, on its first filtered update
        if (!h.filter_scratch) {
            CSK_HIP(hipStreamSynchronize(s));
            if (hipMalloc(&h.filter_scratch, fb) != hipSuccess) {
                h.filter_scratch = nullptr;
                return fail(CS_ENOMEM, "filtered update buffer");
            }
            h.filter_scratch_bytes = fb;
        }
        a.scratch = h.filter_scratch;
        a.scratch_bytes = h.filter_scratch_bytes;
    }
    if (n_kept) {
        a.kept = h.kept_dev;
        st = zero_device_u64(h.kept_dev, s);
        if (st != CS_OK) return st;
    }
    st = launch_update(a, CS_UPDATE_AUTO, 0, s);
    if (st != CS_OK || !n_kept) return st;
    unsigned long long cnt = 0;
    CSK_HIP(hipMemcpyAsync(&cnt, h.kept_dev, sizeof(cnt), hipMemcpyDeviceToHost, s));
    CSK_HIP(hipStreamSynchronize(s));
    *n_kept = cnt;
    return CS_OK;
}

cs_status cs_update(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                    void *stream)
{
    return cs_update_ex(hs, rel, keys, weights, n, stream, CS_UPDATE_AUTO, 0, 0);
}

cs_status cs_estimate(cs_sketch *hs, void *stream, cs_estimate_t *out, const cs_reps_t *reps)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    return estimate_run(hs->h, static_cast<hipStream_t>(stream), out, reps);
}

cs_status cs_estimate_async(cs_sketch *hs, void *stream, cs_estimate_t *out)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    // the result is written by a kernel: refuse memory the device cannot reach (pageable
    // host memory would fault the GPU) before anything is enqueued
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, out) != hipSuccess) {
        (void)hipGetLastError();  // clear the lookup's error for the caller's next call
        return fail(CS_EINVAL, "estimate destination is neither device nor pinned host memory");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeHost && attr.type != hipMemoryTypeManaged)
        return fail(CS_EINVAL, "estimate destination is neither device nor pinned host memory");
    if (attr.type == hipMemoryTypeDevice && attr.device != hs->h.device)
        return fail(CS_EINVAL, "estimate destination on another device");
    return estimate_run_async(hs->h, static_cast<hipStream_t>(stream), out);
}

cs_status cs_reset(cs_sketch *hs, void *stream)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    Handle &h = hs->h;
    const size_t n = (size_t)h.g.n_rel * h.d * h.m;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h.counters, n);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

cs_status cs_merge(cs_sketch *dst, const cs_sketch *src, void *stream)
{
    if (!dst || !src) return fail(CS_EINVAL, "null handle");
    const Handle &a = dst->h, &b = src->h;
    if (a.m != b.m || a.d != b.d || a.seed != b.seed || a.g.attr_rel != b.g.attr_rel || a.g.edges != b.g.edges)
        return fail(CS_EINVAL, "merge needs the same query, m, d and seed");
    const size_t n = (size_t)a.g.n_rel * a.d * a.m;
    hipLaunchKernelGGL(k_add_i64, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dst->h.counters, b.counters, n);
    CSK_HIP(hipGetLastError());
    return CS_OK;
}

cs_status cs_read_sketch(cs_sketch *hs, int32_t rel, int64_t *host_out)
{
    if (!hs || !host_out) return fail(CS_EINVAL, "null argument");
    Handle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    CSK_HIP(hipDeviceSynchronize());
    CSK_HIP(hipMemcpy(host_out, h.counters + (size_t)rel * h.d * h.m, (size_t)h.d * h.m * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    return CS_OK;
}

cs_status cs_timer_create(void **ev)
{
    if (!ev) return fail(CS_EINVAL, "null argument");
    hipEvent_t e = nullptr;
    CSK_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    *ev = e;
    return CS_OK;
}

cs_status cs_timer_record(void *ev, void *stream)
{
    if (!ev) return fail(CS_EINVAL, "null event");
    CSK_HIP(hipEventRecord(static_cast<hipEvent_t>(ev), static_cast<hipStream_t>(stream)));
    return CS_OK;
}

cs_status cs_timer_elapsed(void *start, void *stop, float *ms)
{
    if (!start || !stop || !ms) return fail(CS_EINVAL, "null argument");
    CSK_HIP(hipEventSynchronize(static_cast<hipEvent_t>(stop)));
    CSK_HIP(hipEventElapsedTime(ms, static_cast<hipEvent_t>(start), static_cast<hipEvent_t>(stop)));
    return CS_OK;
}

cs_status cs_timer_destroy(void *ev)
{
    if (!ev) return CS_OK;
    CSK_HIP(hipEventDestroy(static_cast<hipEvent_t>(ev)));
    return CS_OK;
}

cs_status cs_sketch_device_ptr(cs_sketch *hs, int32_t rel, int64_t **out)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    Handle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    *out = h.counters + (size_t)rel * h.d * h.m;
    return CS_OK;
}

cs_status cs_read_coeffs(const cs_sketch *hs, uint64_t *sign_out, uint64_t *bin_out)
{
    if (!hs) return fail(CS_EINVAL, "null handle");
    const Handle &h = hs->h;
    if (sign_out) std::memcpy(sign_out, h.sign_coef.data(), h.sign_coef.size() * sizeof(uint64_t));
    if (bin_out) std::memcpy(bin_out, h.bin_coef.data(), h.bin_coef.size() * sizeof(uint64_t));
    return CS_OK;
}

cs_status cs_read_components(const cs_sketch *hs, int32_t *psi_out)
{
    if (!hs || !psi_out) return fail(CS_EINVAL, "null argument");
    std::memcpy(psi_out, hs->h.g.psi.data(), hs->h.g.psi.size() * sizeof(int32_t));
    return CS_OK;
}

}  // extern "C"
