// Autotuner for the plain update (Alg. 2): for one (device, m, d, key-column shape,
// weight kind, input-size class) it times every applicable kernel variant -- global
// atomics, wave-aggregated atomics, the LDS-segmented kernels at several chunk counts,
// with and without 16-bit counters and the compacting queue, and the partition by
// bucket range -- on the caller's own tuples, checks that each variant's counters equal
// those of the plain global-atomic kernel, and keeps the fastest.  cs_update's automatic
// strategy then takes the tuned choice for that class; the table can be saved to and
// loaded from a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "csk_handle.h"
#include "csk_internal.h"

namespace csk {

namespace {

// scope 0: plain update (cs_update's strategy); 1: a batched update task (kind and
// tuple chunk of k_batch_update's tasks); 2: the split of two-pass transforms of length m.
struct TuneKey {
    std::string arch;  // gcnArchName and compute-unit count
    int32_t scope = 0;
    uint32_t m;
    int32_t d, n_cols, e1, unit, n_class;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(scope, arch, m, d, n_cols, e1, unit, n_class) <
               std::tie(o.scope, o.arch, o.m, o.d, o.n_cols, o.e1, o.unit, o.n_class);
    }
};
struct TuneChoice {
    int32_t strategy, grid, flags;
    float ms;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;
std::map<int, std::string> g_arch;  // device -> arch string

std::string arch_of(int device)
{
    auto it = g_arch.find(device);
    if (it != g_arch.end()) return it->second;
    hipDeviceProp_t p{};
    std::string a = "unknown";
    if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        std::string name(p.gcnArchName);
        const size_t colon = name.find(':');  // drop feature suffixes (":sramecc+:xnack-")
        if (colon != std::string::npos) name = name.substr(0, colon);
        a = name + "-" + std::to_string(p.multiProcessorCount) + "cu";
    }
    g_arch[device] = a;
    return a;
}

int n_class_of(uint64_t n)
{
    int c = 0;
    while ((n >> (c + 1)) != 0) ++c;
    return c;  // floor(log2 n)
}

int scope_of_strategy(int32_t strategy)
{
    if (strategy == CS_TUNE_BATCH_ATOMIC || strategy == CS_TUNE_BATCH_SEGMENT || strategy == CS_TUNE_BATCH_SORT)
        return 1;
    if (strategy == CS_TUNE_TRANSFORM_SPLIT) return 2;
    return 0;
}

TuneKey key_of(const UpdateArgs &a, int device)
{
    TuneKey k;
    k.scope = 0;
    k.arch = arch_of(device);
    k.m = a.m;
    k.d = a.d;
    k.n_cols = a.plan.n_cols;
    bool e1 = true;
    for (int c = 0; c < a.plan.n_cols; ++c) e1 = e1 && a.plan.n_edges[c] == 1;
    k.e1 = e1;
    k.unit = (a.weights == nullptr || a.unit_weights) ? 1 : 0;
    k.n_class = n_class_of(a.n);
    return k;
}

__global__ void k_diff_u64(const uint64_t *__restrict__ x, const uint64_t *__restrict__ y, size_t n,
                           unsigned int *flag)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (x[i] != y[i]) atomicOr(flag, 1u);
}

struct Cand {
    int32_t strategy, grid, flags;
};

}  // namespace

bool tune_lookup(const UpdateArgs &a, int device, int *strategy, int *grid, int *flags)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return false;
    auto it = g_tune.find(key_of(a, device));
    if (it == g_tune.end()) return false;
    *strategy = it->second.strategy;
    *grid = it->second.grid;
    *flags = it->second.flags;
    return true;
}

TuneKey batch_key(int device, uint32_t m, int d, int n_cols, int e1, int unit, uint64_t n)
{
    TuneKey k;
    k.arch = arch_of(device);
    k.scope = 1;
    k.m = m;
    k.d = d;
    k.n_cols = n_cols;
    k.e1 = e1;
    k.unit = unit;
    k.n_class = n_class_of(n);
    return k;
}

TuneKey split_key(int device, int log2m)
{
    TuneKey k;
    k.arch = arch_of(device);
    k.scope = 2;
    k.m = 1u << log2m;
    k.d = 0;
    k.n_cols = 0;
    k.e1 = 0;
    k.unit = 0;
    k.n_class = 0;
    return k;
}

bool tune_lookup_batch(int device, uint32_t m, int d, int n_cols, int e1, int unit, uint64_t n, int *kind,
                       int *chunk_log2)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return false;
    auto it = g_tune.find(batch_key(device, m, d, n_cols, e1, unit, n));
    if (it == g_tune.end()) return false;
    const int32_t code = it->second.strategy;
    *kind = code == CS_TUNE_BATCH_ATOMIC ? 0 : code == CS_TUNE_BATCH_SORT ? 2 : 1;
    *chunk_log2 = it->second.grid;
    return true;
}

void tune_store_batch(int device, uint32_t m, int d, int n_cols, int e1, int unit, uint64_t n, int kind,
                      int chunk_log2, float ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[batch_key(device, m, d, n_cols, e1, unit, n)] =
        TuneChoice{kind == 0 ? CS_TUNE_BATCH_ATOMIC : kind == 2 ? CS_TUNE_BATCH_SORT : CS_TUNE_BATCH_SEGMENT,
                   chunk_log2, 0, ms};
}

int tune_split(int device, int log2m)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return 0;
    auto it = g_tune.find(split_key(device, log2m));
    return it == g_tune.end() ? 0 : it->second.grid;
}

void tune_store_split(int device, int log2m, int S, float ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[split_key(device, log2m)] = TuneChoice{CS_TUNE_TRANSFORM_SPLIT, S, 0, ms};
}

}  // namespace csk

using namespace csk;

extern "C" {

cs_status cs_tune_update(cs_sketch *hs, int32_t rel, const uint32_t *keys, const int64_t *weights, uint64_t n,
                         void *stream, int32_t flags, cs_tune_report *out)
{
    if (!hs || !out) return fail(CS_EINVAL, "null argument");
    Handle &h = hs->h;
    if (rel < 0 || rel >= h.g.n_rel) return fail(CS_EINVAL, "relation out of range");
    if (n == 0 || !keys) return fail(CS_EINVAL, "tuning needs a non-empty key buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int device = 0;
    CSK_HIP(hipGetDevice(&device));
    if (device != h.device) return fail(CS_EINVAL, "handle lives on another device");

    UpdateArgs base;
    base.keys = keys;
    base.weights = weights;
    base.n = n;
    base.coef = h.coef_dev + h.coef_off[rel];
    base.m = h.m;
    base.d = (int32_t)h.d;
    base.plan = h.g.rel[rel];
    base.scratch = nullptr;
    base.scratch_bytes = 0;
    base.unit_weights = (flags & CS_UPDATE_UNIT_WEIGHTS) != 0;
    const bool unit = weights == nullptr || base.unit_weights;
    const bool narrow = unit && n < (1ull << 31);

    // ---- candidates (the reference first)
    std::vector<Cand> cands;
    cands.push_back({CS_UPDATE_GLOBAL_ATOMIC, 0, 0});
    cands.push_back({CS_UPDATE_WAVE_AGGREGATE, 0, 0});
    const uint64_t cells = (uint64_t)h.d * h.m;
    if (narrow && h.m <= (1u << 16) && h.m > (1u << 15) && (h.m % 2) == 0) {
        const SegGeom g16 = seg16_geometry(h.m, (int32_t)h.d, (size_t)-1);
        const int32_t one_round = std::max(1, 256 / g16.segments);
        for (int mult : {1, 2, 3, 4}) cands.push_back({CS_UPDATE_LDS_PRIVATE, one_round * mult, 0});
    }
    {
        const SegGeom g = seg_geometry(h.m, (int32_t)h.d, narrow, (size_t)-1);
        const int32_t one_round = std::max(1, 256 / g.segments);
        const int32_t f16 = CS_UPDATE_NO_COUNTERS16;
        for (int mult : {1, 2}) {
            cands.push_back({CS_UPDATE_LDS_PRIVATE, one_round * mult, f16});
            if (narrow && g.R < h.m && base.plan.n_cols <= 2)
                cands.push_back({CS_UPDATE_LDS_PRIVATE, one_round * mult, f16 | CS_UPDATE_NO_COMPACT});
        }
    }
    if (unit && base.plan.n_cols <= 2) cands.push_back({CS_UPDATE_PARTITION, 0, 0});
    if ((int)cands.size() > CS_TUNE_MAX_CANDIDATES) cands.resize(CS_TUNE_MAX_CANDIDATES);

    // ---- two private counter blocks: the reference's and the candidate's
    uint64_t *ref = nullptr, *tmp = nullptr;
    unsigned int *flag = nullptr;
    if (hipMalloc(&ref, cells * 8) != hipSuccess) return fail(CS_ENOMEM, "tuning buffers");
    if (hipMalloc(&tmp, cells * 8) != hipSuccess || hipMalloc(&flag, sizeof(unsigned int)) != hipSuccess) {
        hipFree(ref);
        if (tmp) hipFree(tmp);
        return fail(CS_ENOMEM, "tuning buffers");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    cs_status st = CS_OK;
    auto cleanup = [&]() {
        hipStreamSynchronize(s);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        hipFree(ref);
        hipFree(tmp);
        hipFree(flag);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(CS_EDEVICE, "tuning events");
    }

    std::memset(out, 0, sizeof(*out));
    out->best = -1;
    float best_ms = 0.0f;
    const unsigned diff_blocks = (unsigned)std::min<uint64_t>((cells + 255) / 256, 4096);
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        const Cand &c = cands[ci];
        cs_tune_candidate &o = out->cand[ci];
        o.strategy = c.strategy;
        o.grid_blocks = c.grid;
        o.flags = c.flags;
        o.valid = 0;
        o.ms = -1.0f;
        UpdateArgs a = base;
        a.compact = (c.flags & CS_UPDATE_NO_COMPACT) == 0;
        a.counters16 = (c.flags & CS_UPDATE_NO_COUNTERS16) == 0;
        uint64_t *dst = ci == 0 ? ref : tmp;
        a.sketch = dst;
        // one run from zero, checked against the reference
        if (hipMemsetAsync(dst, 0, cells * 8, s) != hipSuccess) {
            st = fail(CS_EDEVICE, "tuning: clear");
            break;
        }
        if (launch_update(a, c.strategy, c.grid, s) != CS_OK) {
            if (ci == 0) {  // the reference must run
                st = CS_EDEVICE;
                break;
            }
            continue;  // not applicable to this handle
        }
        unsigned int hflag = 0;
        if (ci > 0) {
            if (hipMemsetAsync(flag, 0, sizeof(unsigned int), s) != hipSuccess) {
                st = fail(CS_EDEVICE, "tuning: clear flag");
                break;
            }
            hipLaunchKernelGGL(k_diff_u64, dim3(diff_blocks), dim3(256), 0, s, tmp, ref, cells, flag);
            if (hipMemcpyAsync(&hflag, flag, sizeof(unsigned int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = fail(CS_EDEVICE, "tuning: compare");
                break;
            }
            if (hflag) {  // counters differ from the reference: never chosen
                o.valid = -1;
                continue;
            }
        }
        // timed: median of three runs, adding into the candidate buffer (never the
        // reference's, which the later candidates are checked against)
        a.sketch = tmp;
        float t[3];
        bool ok = true;
        for (int r = 0; r < 3 && ok; ++r) {
            ok = hipEventRecord(e0, s) == hipSuccess && launch_update(a, c.strategy, c.grid, s) == CS_OK &&
                 hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        }
        if (!ok) continue;
        std::sort(t, t + 3);
        o.ms = t[1];
        o.valid = 1;
        if (out->best < 0 || o.ms < best_ms) {
            out->best = (int32_t)ci;
            best_ms = o.ms;
        }
    }
    out->n = (int32_t)cands.size();
    cleanup();
    if (st != CS_OK) return st;
    if (out->best < 0) return fail(CS_EDEVICE, "tuning: no candidate ran");
    const cs_tune_candidate &b = out->cand[out->best];
    UpdateArgs a = base;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key_of(a, device)] = TuneChoice{b.strategy, b.grid_blocks, b.flags, b.ms};
    return CS_OK;
}

cs_status cs_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return CS_OK;
}

cs_status cs_tune_save(const char *path)
{
    if (!path) return fail(CS_EINVAL, "null path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(CS_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "csketch-tune 1\n");
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const TuneChoice &c = kv.second;
        std::fprintf(f, "%s %u %d %d %d %d %d %d %d %d %.6f\n", k.arch.c_str(), k.m, k.d, k.n_cols, k.e1, k.unit,
                     k.n_class, c.strategy, c.grid, c.flags, c.ms);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? CS_OK : fail(CS_EINVAL, std::string("cannot write ") + path);
}

cs_status cs_tune_load(const char *path)
{
    if (!path) return fail(CS_EINVAL, "null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(CS_EINVAL, std::string("cannot read ") + path);
    char line[512];
    std::map<TuneKey, TuneChoice> got;
    bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, "csketch-tune 1", 14) == 0;
    while (ok && std::fgets(line, sizeof line, f)) {
        if (line[0] == '\n' || line[0] == '#') continue;
        char arch[128];
        TuneKey k;
        TuneChoice c;
        const int nf = std::sscanf(line, "%127s %u %d %d %d %d %d %d %d %d %f", arch, &k.m, &k.d, &k.n_cols, &k.e1,
                                   &k.unit, &k.n_class, &c.strategy, &c.grid, &c.flags, &c.ms);
        k.scope = scope_of_strategy(c.strategy);
        if (nf != 11) {
            ok = false;
        } else if (k.scope == 0) {
            ok = c.strategy > CS_UPDATE_AUTO && c.strategy <= CS_UPDATE_PARTITION && k.d >= 1 && k.d <= kMaxD &&
                 k.m >= 1 && c.grid >= 0;
        } else if (k.scope == 1) {  // grid: log2 of the tuples per task
            ok = k.d >= 1 && k.d <= kMaxD && k.m >= 1 && c.grid >= 12 && c.grid <= 22;
        } else {  // grid: log2 of the row length of the two-pass transform of length m
            const bool pow2 = k.m >= 2 && (k.m & (k.m - 1)) == 0;
            const int L = pow2 ? 31 - __builtin_clz(k.m) : 0;
            ok = pow2 && L > 12 && L <= kMaxLog2N && split_ok(L, c.grid);
        }
        if (ok) {
            k.arch = arch;
            got[k] = c;
        }
    }
    std::fclose(f);
    if (!ok) return fail(CS_EINVAL, std::string("malformed tuning file ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : got) g_tune[kv.first] = kv.second;
    return CS_OK;
}

cs_status cs_tune_count(int32_t *n_out)
{
    if (!n_out) return fail(CS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *n_out = (int32_t)g_tune.size();
    return CS_OK;
}

}  // extern "C"
