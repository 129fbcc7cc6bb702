// ann_search_noalloc: the batched search of ann_search with its scratch
// memory (the persistent launch's work counter and the widest-first query
// order with its keys) held in a fixed device array of this library instead
// of a caller workspace, for callers that cannot allocate.
#include <mutex>

#include "internal.h"

using namespace ann;

namespace {

constexpr int kMaxDevices = 64;

// counter (256 bytes), then the order and its keys (4 bytes each per query),
// exactly the layout ann_search carves from its workspace
constexpr size_t kScratchBytes = 256 + 2 * (((size_t)ANN_NOALLOC_MAX_QUERIES * 4 + 255) / 256 * 256);

// One copy per GPU, kept until the process ends.  Host code never passes
// this name to a kernel: it uses the device address from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
ann_status scratch_on_current_device(void **out)
{
    int dev = -1;
    ANN_HIP(hipGetDevice(&dev));
    ANN_SUPPORTED(dev >= 0 && dev < kMaxDevices, "device %d beyond the %d this library tracks", dev,
                  kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        ANN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        ANN_REQUIRE(p != nullptr, "hipGetSymbolAddress returned NULL for the scratch array");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return ANN_OK;
}

}  // namespace

extern "C" ann_status ann_search_noalloc(const float *base, int64_t n, int32_t dim,
                                         const int32_t *graph, int32_t R, const float *queries,
                                         int32_t nq, const int32_t *entry_ids, int32_t medoid,
                                         const int32_t *k, const int32_t *L, int32_t k_max,
                                         int32_t *out_ids, float *out_dist, int32_t *stats,
                                         int32_t *trace, int32_t trace_cap,
                                         const ann_search_plan *plan, void *stream)
{
    ANN_REQUIRE(nq >= 0 && nq <= ANN_NOALLOC_MAX_QUERIES,
                "ann_search_noalloc takes at most %d queries per call (got %d)",
                ANN_NOALLOC_MAX_QUERIES, nq);
    void *ws = nullptr;
    ann_status s = scratch_on_current_device(&ws);
    if (s != ANN_OK) return s;
    ann_search_plan p{};
    s = search_check(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L, k_max, out_ids,
                     out_dist, trace, trace_cap, plan, ws, kScratchBytes, p);
    if (s != ANN_OK) return s;
    if (nq == 0) return ANN_OK;
    return search_launch(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L, k_max,
                         out_ids, out_dist, stats, trace, trace_cap, p, static_cast<uint32_t *>(ws),
                         static_cast<hipStream_t>(stream), true);
}
