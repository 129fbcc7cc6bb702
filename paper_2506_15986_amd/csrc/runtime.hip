// Batch driver around the search and entry-selection kernels: candidate
// plans and their timing (the autotuner), one-call batches of the query path
// (entry selection, then the persistent search launch) and HIP graphs of
// those batches.
#include "common.h"
#include "internal.h"

#include <hip/hip_ext.h>

#include <new>
#include <vector>

namespace ann {
namespace {

__global__ void tune_copy_kernel(const int32_t *ids, const float *dist, int64_t count,
                                 int32_t *ref_ids, float *ref_dist)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    ref_ids[i] = ids[i];
    ref_dist[i] = dist[i];
}

__global__ void tune_zero_kernel(uint32_t *p) { *p = 0u; }

// counts positions whose id or distance bits differ from the reference
__global__ void tune_compare_kernel(const int32_t *ids, const float *dist, int64_t count,
                                    const int32_t *ref_ids, const float *ref_dist, uint32_t *bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (ids[i] != ref_ids[i] || __float_as_uint(dist[i]) != __float_as_uint(ref_dist[i]))
        atomicAdd(bad, 1u);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

// one reference result per gather group (4, 8, 16)
size_t autotune_ws(int64_t n, int dim, int nq, int k_max)
{
    size_t b = round_up(ann_workspace_size(ANN_OP_SEARCH, n, dim, nq, 0), 256);
    b += round_up((size_t)nq * k_max * 4, 256) * 6;
    b += 256;
    return b;
}

ann_status query_run(const ann_query_batch &b, int stages, hipStream_t st)
{
    ANN_REQUIRE(stages >= 1 && stages <= ANN_STAGE_ALL, "stages must be a non-empty ANN_STAGE_* set");
    ann_search_plan p{};
    if (stages & ANN_STAGE_SEARCH) {
        ann_status s = search_check(b.base, b.n, b.dim, b.graph, b.R, b.queries, b.nq,
                                    b.entry_ids, b.medoid, b.k, b.L, b.k_max, b.out_ids,
                                    b.out_dist, nullptr, 0, &b.plan, b.search_ws,
                                    b.search_ws_bytes, p);
        if (s != ANN_OK) return s;
    }
    if (stages & ANN_STAGE_ENTRY) {
        ANN_REQUIRE(b.model != nullptr && b.entry_ids != nullptr,
                    "the entry stage needs a model and an entry_ids buffer");
        ann_status s = ann_entry_select(b.model, b.queries, b.nq, b.dim, b.entry_ids, nullptr,
                                        nullptr, b.entry_ws, b.entry_ws_bytes, st);
        if (s != ANN_OK) return s;
    }
    if ((stages & ANN_STAGE_SEARCH) && b.nq > 0)
        return search_launch(b.base, b.n, b.dim, b.graph, b.R, b.queries, b.nq, b.entry_ids,
                             b.medoid, b.k, b.L, b.k_max, b.out_ids, b.out_dist, b.stats,
                             nullptr, 0, p, static_cast<uint32_t *>(b.search_ws), st, true);
    return ANN_OK;
}

}  // namespace ann

using namespace ann;

struct ann_query_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ann_query_batch batch{};
    ann_entry_model model{};
};

extern "C" int32_t ann_autotune_candidates(int64_t n, int32_t dim, int32_t R, int32_t L_max,
                                           ann_search_plan *plans, int32_t cap)
{
    if (n < 1 || dim < 1 || R < 1 || L_max < 1 || L_max > 1024) return 0;
    ann_search_plan base{};
    if (ann_default_plan(n, dim, R, L_max, &base) != ANN_OK) return 0;
    std::vector<ann_search_plan> out;
    out.push_back(base);    // the default plan first: the reference for the result check
    const int groups[3] = {4, 8, 16};
    for (int g : groups) {
        if (g == 4 && dim > 64) continue;
        if (g == 8 && dim > 128) continue;
        for (int vl = 10; vl <= 13; ++vl) {
            for (int wpb = 1; wpb <= 4; wpb *= 2) {
                ann_search_plan p = base;
                p.group = g;
                p.visited_log2 = vl;
                p.waves_per_block = wpb;
                if (p.group == base.group && p.visited_log2 == base.visited_log2 &&
                    p.waves_per_block == base.waves_per_block)
                    continue;
                if (search_wave_lds(p, n, dim) == 0) continue;
                out.push_back(p);
            }
            if (g != 16) continue;
            for (int wq = 2; wq <= 4; wq *= 2) {
                ann_search_plan p = base;
                p.group = 16;
                p.visited_log2 = vl;
                p.waves_per_query = wq;
                p.waves_per_block = wq;
                if (search_wave_lds(p, n, dim) == 0) continue;
                out.push_back(p);
            }
        }
    }
    const int32_t total = (int32_t)out.size();
    if (plans)
        for (int32_t i = 0; i < total && i < cap; ++i) plans[i] = out[i];
    return total;
}

extern "C" size_t ann_autotune_workspace_size(int64_t n, int32_t dim, int32_t nq, int32_t k_max)
{
    return autotune_ws(n, dim, nq, k_max);
}

extern "C" ann_status ann_autotune_search(const float *base, int64_t n, int32_t dim,
                                          const int32_t *graph, int32_t R, const float *queries,
                                          int32_t nq, const int32_t *entry_ids, int32_t medoid,
                                          const int32_t *k, const int32_t *L, int32_t k_max,
                                          int32_t *out_ids, float *out_dist, int32_t *stats,
                                          const ann_search_plan *cands, int32_t n_cand,
                                          int32_t reps, ann_search_plan *best, float *times_ms,
                                          void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(cands && best && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n_cand >= 1, "n_cand must be >= 1");
    ANN_REQUIRE(reps >= 1, "reps must be >= 1");
    ANN_REQUIRE(nq >= 1, "the tuning batch must hold at least one query");
    ANN_REQUIRE(ws_bytes >= autotune_ws(n, dim, nq, k_max), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    const size_t sws = ann_workspace_size(ANN_OP_SEARCH, n, dim, nq, 0);
    void *search_ws = cv.take<unsigned char>(sws);
    const int64_t cells = (int64_t)nq * k_max;
    int32_t *ref_ids[3];
    float *ref_dist[3];
    for (int r = 0; r < 3; ++r) {
        ref_ids[r] = cv.take<int32_t>((size_t)cells);
        ref_dist[r] = cv.take<float>((size_t)cells);
    }
    uint32_t *bad = cv.take<uint32_t>(64);
    // every candidate is checked on the host before any work is enqueued
    std::vector<ann_search_plan> plans(cands, cands + n_cand);
    std::vector<int> runs(n_cand, 0);
    int n_run = 0;
    for (int c = 0; c < n_cand; ++c) {
        ann_search_plan p{};
        ann_status s = search_check(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L,
                                    k_max, out_ids, out_dist, nullptr, 0, &plans[c], search_ws,
                                    sws, p);
        if (s == ANN_EINVAL) return s;
        runs[c] = s == ANN_OK;
        n_run += runs[c];
        if (times_ms) times_ms[c] = -1.0f;
    }
    ANN_SUPPORTED(n_run > 0, "no candidate plan fits this index on the device");
    EventPair ev;
    ANN_HIP(hipEventCreate(&ev.a));
    ANN_HIP(hipEventCreate(&ev.b));
    // plans with the same gather group sum every distance in the same order,
    // so their results must agree bit for bit; across groups the FP32 order
    // differs (exact data aside), so each group is checked against its first
    int first[3] = {-1, -1, -1}, bestc = -1;
    float best_ms = 0.0f;
    for (int c = 0; c < n_cand; ++c) {
        if (!runs[c]) continue;
        ann_status s = search_launch(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L,
                                     k_max, out_ids, out_dist, stats, nullptr, 0, plans[c],
                                     static_cast<uint32_t *>(search_ws), st, true);
        if (s != ANN_OK) return s;
        ANN_HIP(hipEventRecord(ev.a, st));
        for (int r = 0; r < reps; ++r) {
            s = search_launch(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L, k_max,
                              out_ids, out_dist, stats, nullptr, 0, plans[c],
                              static_cast<uint32_t *>(search_ws), st, true);
            if (s != ANN_OK) return s;
        }
        ANN_HIP(hipEventRecord(ev.b, st));
        ANN_HIP(hipEventSynchronize(ev.b));
        float ms = 0.0f;
        ANN_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        ms /= (float)reps;
        if (times_ms) times_ms[c] = ms;
        const int gi = plans[c].group == 4 ? 2 : plans[c].group == 8 ? 0 : 1;
        if (first[gi] < 0) {
            first[gi] = c;
            hipLaunchKernelGGL(tune_copy_kernel, dim3(grid_for(cells)), dim3(256), 0, st, out_ids,
                               out_dist, cells, ref_ids[gi], ref_dist[gi]);
            ANN_LAUNCHED();
        } else {
            hipLaunchKernelGGL(tune_zero_kernel, dim3(1), dim3(1), 0, st, bad);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(tune_compare_kernel, dim3(grid_for(cells)), dim3(256), 0, st,
                               out_ids, out_dist, cells, ref_ids[gi], ref_dist[gi], bad);
            ANN_LAUNCHED();
            uint32_t nbad = 0;
            ANN_HIP(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, st));
            ANN_HIP(hipStreamSynchronize(st));
            if (nbad != 0)
                return fail(ANN_EDEVICE,
                            "plan %d (group %d, visited_log2 %d, waves_per_block %d) differs from "
                            "plan %d in %u result cells",
                            c, plans[c].group, plans[c].visited_log2, plans[c].waves_per_block,
                            first[gi], nbad);
        }
        if (bestc < 0 || ms < best_ms) {
            bestc = c;
            best_ms = ms;
        }
    }
    ANN_HIP(hipStreamSynchronize(st));
    *best = plans[bestc];
    return ANN_OK;
}

extern "C" ann_status ann_query_run(const ann_query_batch *batch, int32_t stages, void *stream)
{
    ANN_REQUIRE(batch != nullptr, "batch is NULL");
    return query_run(*batch, stages, static_cast<hipStream_t>(stream));
}

extern "C" ann_status ann_query_graph_create(const ann_query_batch *batch, int32_t stages,
                                             ann_query_graph **out)
{
    ANN_REQUIRE(batch != nullptr && out != nullptr, "a required pointer is NULL");
    *out = nullptr;
    ANN_REQUIRE(stages >= 1 && stages <= ANN_STAGE_ALL, "stages must be a non-empty ANN_STAGE_* set");
    ann_query_graph *g = new (std::nothrow) ann_query_graph();
    ANN_REQUIRE(g != nullptr, "out of host memory");
    g->batch = *batch;
    if (batch->model) {
        g->model = *batch->model;
        g->batch.model = &g->model;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return fail(ANN_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    ann_status s = ANN_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        s = fail(ANN_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    } else {
        s = query_run(g->batch, stages, cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (s == ANN_OK && e != hipSuccess)
            s = fail(ANN_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        g->graph = graph;
    }
    (void)hipStreamDestroy(cs);
    if (s == ANN_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) s = fail(ANN_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (s != ANN_OK) {
        ann_query_graph_destroy(g);
        return s;
    }
    *out = g;
    return ANN_OK;
}

extern "C" ann_status ann_query_graph_launch(ann_query_graph *graph, void *stream)
{
    ANN_REQUIRE(graph != nullptr && graph->exec != nullptr, "graph is NULL");
    ANN_HIP(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
    return ANN_OK;
}

extern "C" void ann_query_graph_destroy(ann_query_graph *graph)
{
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

extern "C" ann_status ann_stream_create(void **out)
{
    ANN_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int dev = 0, cus = 0;
    ANN_HIP(hipGetDevice(&dev));
    ANN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus <= 0) return fail(ANN_EDEVICE, "device reports %d compute units", cus);
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xFFFFFFFFu);
    if (cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
    hipStream_t st = nullptr;
    ANN_HIP(hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()));
    *out = st;
    return ANN_OK;
}

extern "C" void ann_stream_destroy(void *stream)
{
    if (stream) (void)hipStreamDestroy(static_cast<hipStream_t>(stream));
}
