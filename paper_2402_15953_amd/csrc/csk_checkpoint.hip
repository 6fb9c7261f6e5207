// Checkpoint and resume of a sketch handle.  A sketch is its counters plus what draws
// its hash functions (the query graph, m, d and the seed; Sec. 2.5 counts exactly these
// in a sketch's memory), so an exported blob re-creates an identical handle, and sketch
// linearity (Sec. 2.2) makes "import, then keep updating" equal to never stopping.
//
// Blob layout (little-endian): "CSKETCH1", uint32 version = 1, m, d, n_rel, n_attr,
// n_edge, uint64 seed, int32 attr_rel[n_attr], int32 edges[n_edge][2],
// int64 counters[n_rel][d][m], uint64 FNV-1a of every preceding byte.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "csk_handle.h"
#include "csk_internal.h"

namespace csk {
namespace {

constexpr char kMagic[8] = {'C', 'S', 'K', 'E', 'T', 'C', 'H', '1'};
constexpr uint32_t kVersion = 1;

uint64_t fnv1a(const unsigned char *p, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

size_t blob_bytes(uint32_t n_attr, uint32_t n_edge, uint64_t n_counters)
{
    return 8 + 6 * 4 + 8 + (size_t)n_attr * 4 + (size_t)n_edge * 8 + n_counters * 8 + 8;
}

template <typename T>
void put(unsigned char *&p, T v)
{
    std::memcpy(p, &v, sizeof(T));
    p += sizeof(T);
}

template <typename T>
T get(const unsigned char *&p)
{
    T v;
    std::memcpy(&v, p, sizeof(T));
    p += sizeof(T);
    return v;
}

}  // namespace
}  // namespace csk

using namespace csk;

extern "C" {

cs_status cs_export(cs_sketch *hs, void *buf, size_t cap, size_t *needed)
{
    if (!hs || !needed) return fail(CS_EINVAL, "null argument");
    const Handle &h = hs->h;
    const uint64_t nc = (uint64_t)h.g.n_rel * h.d * h.m;
    const size_t total = blob_bytes((uint32_t)h.g.n_attr, (uint32_t)h.g.n_edge, nc);
    *needed = total;
    if (!buf) return CS_OK;
    if (cap < total) return fail(CS_EINVAL, "export buffer too small");
    unsigned char *p = static_cast<unsigned char *>(buf);
    std::memcpy(p, kMagic, 8);
    p += 8;
    put<uint32_t>(p, kVersion);
    put<uint32_t>(p, h.m);
    put<uint32_t>(p, h.d);
    put<uint32_t>(p, (uint32_t)h.g.n_rel);
    put<uint32_t>(p, (uint32_t)h.g.n_attr);
    put<uint32_t>(p, (uint32_t)h.g.n_edge);
    put<uint64_t>(p, h.seed);
    for (int32_t v : h.g.attr_rel) put<int32_t>(p, v);
    for (int32_t v : h.g.edges) put<int32_t>(p, v);
    CSK_HIP(hipDeviceSynchronize());
    CSK_HIP(hipMemcpy(p, h.counters, nc * sizeof(int64_t), hipMemcpyDeviceToHost));
    p += nc * sizeof(int64_t);
    const unsigned char *base = static_cast<unsigned char *>(buf);
    put<uint64_t>(p, fnv1a(base, (size_t)(p - base)));
    return CS_OK;
}

cs_status cs_import(const void *buf, size_t len, cs_sketch **out)
{
    if (!buf || !out) return fail(CS_EINVAL, "null argument");
    *out = nullptr;
    const unsigned char *base = static_cast<const unsigned char *>(buf);
    const size_t head = 8 + 6 * 4 + 8;
    if (len < head + 8 || std::memcmp(base, kMagic, 8) != 0) return fail(CS_EINVAL, "not a sketch checkpoint");
    const unsigned char *p = base + 8;
    const uint32_t version = get<uint32_t>(p);
    const uint32_t m = get<uint32_t>(p), d = get<uint32_t>(p);
    const uint32_t n_rel = get<uint32_t>(p), n_attr = get<uint32_t>(p), n_edge = get<uint32_t>(p);
    const uint64_t seed = get<uint64_t>(p);
    if (version != kVersion) return fail(CS_EINVAL, "unsupported checkpoint version");
    if (m < 2 || m > (1u << kMaxLog2M) || d < 1 || d > (uint32_t)kMaxD || n_rel < 1 || n_attr < 1 ||
        n_attr > 4096 || n_edge > 4096)
        return fail(CS_EINVAL, "checkpoint header out of range");
    const uint64_t nc = (uint64_t)n_rel * d * m;
    if (len != blob_bytes(n_attr, n_edge, nc)) return fail(CS_EINVAL, "checkpoint length mismatch");
    uint64_t stored;
    std::memcpy(&stored, base + len - 8, 8);
    if (stored != fnv1a(base, len - 8)) return fail(CS_EINVAL, "checkpoint checksum mismatch");
    std::vector<int32_t> attr_rel(n_attr), edges((size_t)n_edge * 2);
    for (auto &v : attr_rel) v = get<int32_t>(p);
    for (auto &v : edges) v = get<int32_t>(p);
    cs_graph g{(int32_t)n_rel, (int32_t)n_attr, attr_rel.data(), (int32_t)n_edge, edges.data()};
    cs_sketch *hs = nullptr;
    cs_status st = create_handle(&g, m, d, seed, true, &hs);
    if (st != CS_OK) return st;
    if (hipMemcpy(hs->h.counters, p, nc * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
        cs_destroy(hs);
        return fail(CS_EDEVICE, "checkpoint upload failed");
    }
    *out = hs;
    return CS_OK;
}

}  // extern "C"
