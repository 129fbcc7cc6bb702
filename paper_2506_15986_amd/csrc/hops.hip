// Hop counts of Definition 4: H(q, V_h), the length of the shortest path
// along the graph's edges from hub h to the nearest neighbour of query q.
//
// Hubs run 64 at a time as the bits of one 64-bit word per node (a
// multi-source breadth-first search).  Each level, every node on the
// frontier ORs its hub bits into its out-neighbours' next words, minus the
// bits they have already seen; the bits a node gains form its frontier for
// the next level.  After level l, a query whose target gained bit b gets
// H = l for hub (first + b).  Every H starts at 255 (unreachable, or more
// than 254 hops).
#include <vector>

#include "common.h"
#include "internal.h"

namespace ann {
namespace {

using u64 = unsigned long long;

__global__ void hops_fill_kernel(uint8_t *p, int64_t count, uint8_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void hops_zero_kernel(u64 *p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// level 0: hub (first + b) holds bit b
__global__ void hops_seed_kernel(const int32_t *hubs, int first, int nb, u64 *seen, u64 *front)
{
    const int b = threadIdx.x;
    if (b >= nb) return;
    const int32_t v = hubs[first + b];
    atomicOr(&seen[v], 1ull << b);
    atomicOr(&front[v], 1ull << b);
}

__global__ void hops_expand_kernel(const int32_t *graph, int64_t n, int R, const u64 *front,
                                   const u64 *seen, u64 *next)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const u64 f = front[v];
        if (!f) continue;
        for (int s = 0; s < R; ++s) {
            const int32_t w = graph[v * R + s];
            if (w < 0 || (int64_t)w >= n) continue;
            const u64 add = f & ~seen[w];
            if (add) atomicOr(&next[w], add);
        }
    }
}

// H[q][first + b] = level for every bit b that q's target gained this level
__global__ void hops_record_kernel(const int32_t *targets, int64_t nq, const u64 *gained,
                                   int first, int nh, int level, uint8_t *H)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
         q += (int64_t)gridDim.x * blockDim.x) {
        u64 g = gained[targets[q]];
        while (g) {
            const int b = __builtin_ctzll(g);
            g &= g - 1;
            H[q * nh + first + b] = (uint8_t)level;
        }
    }
}

// the gained bits become the frontier and join the seen bits
__global__ void hops_settle_kernel(int64_t n, u64 *seen, u64 *front, u64 *next, int32_t *any)
{
    int local = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const u64 x = next[v];
        front[v] = x;
        if (x) {
            seen[v] |= x;
            next[v] = 0ull;
            local = 1;
        }
    }
    if (local) atomicOr(any, 1);
}

__global__ void hops_flag_reset_kernel(int32_t *any) { *any = 0; }

inline int hop_grid(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

size_t hop_ws(int64_t n) { return round_up((size_t)n * 8, 256) * 3 + 256; }

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" size_t ann_hop_table_workspace_size(int64_t n)
{
    return n >= 1 ? hop_ws(n) : 0;
}

extern "C" ann_status ann_hop_table(const int32_t *graph, int64_t n, int32_t R, const int32_t *hub_ids,
                                    int32_t n_hubs, const int32_t *targets, int64_t nq, uint8_t *out,
                                    void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(graph && hub_ids && workspace, "a required pointer is NULL");
    ANN_REQUIRE(nq == 0 || (targets && out), "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(R >= 1, "R must be >= 1");
    ANN_REQUIRE(n_hubs >= 1, "n_hubs must be >= 1");
    ANN_REQUIRE(nq >= 0, "nq must be >= 0");
    ANN_REQUIRE(ws_bytes >= hop_ws(n), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // host check of the hub and target ids (the kernels index with them)
    {
        std::vector<int32_t> h((size_t)n_hubs);
        ANN_HIP(hipMemcpyAsync(h.data(), hub_ids, sizeof(int32_t) * (size_t)n_hubs,
                               hipMemcpyDeviceToHost, st));
        std::vector<int32_t> t((size_t)nq);
        if (nq)
            ANN_HIP(hipMemcpyAsync(t.data(), targets, sizeof(int32_t) * (size_t)nq,
                                   hipMemcpyDeviceToHost, st));
        ANN_HIP(hipStreamSynchronize(st));
        for (int32_t v : h) ANN_REQUIRE(v >= 0 && (int64_t)v < n, "hub id %d out of range", v);
        for (int32_t v : t) ANN_REQUIRE(v >= 0 && (int64_t)v < n, "target id %d out of range", v);
    }
    if (nq == 0) return ANN_OK;
    Carve cv{static_cast<unsigned char *>(workspace)};
    u64 *seen = cv.take<u64>((size_t)n);
    u64 *front = cv.take<u64>((size_t)n);
    u64 *next = cv.take<u64>((size_t)n);
    int32_t *any = cv.take<int32_t>(64);
    const int gn = hop_grid(n), gq = hop_grid(nq);
    hipLaunchKernelGGL(hops_fill_kernel, dim3(hop_grid(nq * n_hubs)), dim3(256), 0, st, out,
                       nq * n_hubs, (uint8_t)255);
    ANN_LAUNCHED();
    for (int first = 0; first < n_hubs; first += 64) {
        const int nb = n_hubs - first < 64 ? n_hubs - first : 64;
        for (u64 *p : {seen, front, next}) {
            hipLaunchKernelGGL(hops_zero_kernel, dim3(gn), dim3(256), 0, st, p, n);
            ANN_LAUNCHED();
        }
        hipLaunchKernelGGL(hops_seed_kernel, dim3(1), dim3(64), 0, st, hub_ids, first, nb, seen, front);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(hops_record_kernel, dim3(gq), dim3(256), 0, st, targets, nq, seen, first,
                           n_hubs, 0, out);
        ANN_LAUNCHED();
        for (int level = 1; level <= 254; ++level) {
            hipLaunchKernelGGL(hops_expand_kernel, dim3(gn), dim3(256), 0, st, graph, n, R, front, seen,
                               next);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(hops_record_kernel, dim3(gq), dim3(256), 0, st, targets, nq, next, first,
                               n_hubs, level, out);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(hops_flag_reset_kernel, dim3(1), dim3(1), 0, st, any);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(hops_settle_kernel, dim3(gn), dim3(256), 0, st, n, seen, front, next, any);
            ANN_LAUNCHED();
            int32_t h = 0;
            ANN_HIP(hipMemcpyAsync(&h, any, sizeof(h), hipMemcpyDeviceToHost, st));
            ANN_HIP(hipStreamSynchronize(st));
            if (!h) break;
        }
    }
    return ANN_OK;
}
