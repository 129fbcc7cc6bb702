// Training labels for the entry model: for each historical query, the
// candidate hub from which the plain beam search reaches the target recall
// with the fewest distance computations.
//
// This takes the place of the paper's hop-count queues (Definition 4 and the
// query-aware sample generation, which runs Algorithm 1 from every hub for
// every historical query) with the same intent: which hub serves a query
// best.  For candidate hub m of query q and each beam width L of an
// increasing ladder, the batched beam search (the ann_search kernel) runs from
// that hub; the cost of (q, m) is the distance count of the first width whose
// top-kt holds at least `hits` of the query's true top-kt.  The label is the
// candidate of least cost (ties: smaller hub index), or the first candidate
// when none reaches the target.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

__global__ void gather_entries_kernel(const int32_t *cand, int M, int m, const int32_t *hub_ids,
                                      int nq, int32_t *ent, int32_t *kk, int32_t *LL, int kv, int Lv)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    ent[q] = hub_ids[cand[(int64_t)q * M + m]];
    kk[q] = kv;
    LL[q] = Lv;
}

__global__ void fill_value_kernel(int32_t *p, int64_t count, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// cost of (q, m) at this width if the target is reached for the first time
__global__ void score_kernel(const int32_t *ids, const int32_t *stats, const int32_t *truth,
                             int kt, int hits, int nq, int M, int m, int32_t *table,
                             int32_t *flags)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    int32_t *cell = table + (int64_t)q * M + m;
    if (*cell >= 0) return;
    int h = 0;
    for (int a = 0; a < kt; ++a) {
        const int32_t id = ids[(int64_t)q * kt + a];
        for (int b = 0; b < kt; ++b)
            if (truth[(int64_t)q * kt + b] == id) {
                ++h;
                break;
            }
    }
    const int32_t *st = stats + (int64_t)q * 4;
    if (h >= hits) *cell = st[0];
    if (flags && (st[3] & 1)) flags[q] |= 1;
}

__global__ void choose_kernel(const int32_t *table, const int32_t *cand, int nq, int M,
                              int32_t *labels)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    int32_t best = -1, bh = 0x7fffffff;
    for (int m = 0; m < M; ++m) {
        const int32_t v = table[(int64_t)q * M + m];
        const int32_t h = cand[(int64_t)q * M + m];
        if (v < 0) continue;
        if (best < 0 || v < best || (v == best && h < bh)) {
            best = v;
            bh = h;
        }
    }
    labels[q] = best >= 0 ? bh : cand[(int64_t)q * M];
}

// queries whose searches overflowed the visited table are searched again
// with a table twice as large: their table rows restart, the others get an
// empty width (k = L = 0: the search kernel skips such a row)
__global__ void redo_mark_kernel(int32_t *flags, int nq, int M, int32_t *table, int32_t *redo)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const bool r = (flags[q] & 1) != 0;
    redo[q] = r ? 1 : 0;
    if (r) {
        flags[q] = 0;
        for (int m = 0; m < M; ++m) table[(int64_t)q * M + m] = -1;
    }
}

__global__ void gather_redo_kernel(const int32_t *cand, int M, int m, const int32_t *hub_ids,
                                   const int32_t *redo, int nq, int32_t *ent, int32_t *kk,
                                   int32_t *LL, int kv, int Lv)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    ent[q] = hub_ids[cand[(int64_t)q * M + m]];
    kk[q] = redo[q] ? kv : 0;
    LL[q] = redo[q] ? Lv : 0;
}

__global__ void count_kernel(const int32_t *v, int nq, int32_t *out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq && v[q]) atomicAdd(out, 1);
}

inline int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

size_t make_labels_ws(int nq, int M, int kt)
{
    size_t b = round_up((size_t)nq * 4, 256) * 3;              // entries, k, L
    b += round_up((size_t)nq * kt * 4, 256) * 2;               // ids, dist
    b += round_up((size_t)nq * 16, 256);                       // stats
    b += round_up((size_t)nq * M * 4, 256);                    // table (when not given)
    b += round_up((size_t)nq * 4, 256) * 2;                    // flags (when not given), redo
    b += 512;
    return b;
}

}  // namespace ann

using namespace ann;

extern "C" size_t ann_labels_workspace_size(int32_t nq, int32_t M, int32_t kt)
{
    return make_labels_ws(nq, M, kt);
}

extern "C" ann_status ann_make_labels(const float *base, int64_t n, int32_t dim,
                                      const int32_t *graph, int32_t R, const float *queries,
                                      int32_t nq, const int32_t *truth, int32_t kt, int32_t hits,
                                      const int32_t *cand_hubs, int32_t M, const int32_t *hub_ids,
                                      const int32_t *L_ladder, int32_t n_L, int32_t *labels,
                                      int32_t *table, int32_t *flags, void *workspace,
                                      size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && graph && workspace && L_ladder, "a required pointer is NULL");
    ANN_REQUIRE(nq == 0 || (queries && truth && cand_hubs && hub_ids && labels),
                "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_SUPPORTED(dim % 4 == 0 && dim <= 1024, "dim must be a multiple of 4 and <= 1024");
    ANN_REQUIRE(R >= 1, "R must be >= 1");
    ANN_SUPPORTED(R <= 64, "R must be <= 64");
    ANN_REQUIRE(kt >= 1 && kt <= 64, "kt must be in [1, 64]");
    ANN_REQUIRE(hits >= 1 && hits <= kt, "hits must be in [1, kt]");
    ANN_REQUIRE(M >= 1, "M must be >= 1");
    ANN_REQUIRE(n_L >= 1 && n_L <= 64, "the ladder must hold 1..64 widths");
    for (int i = 0; i < n_L; ++i) {
        ANN_REQUIRE(L_ladder[i] >= kt && L_ladder[i] <= 512, "ladder widths must be in [kt, 512]");
        ANN_REQUIRE(i == 0 || L_ladder[i] > L_ladder[i - 1], "ladder must increase");
    }
    ANN_REQUIRE(aligned(base, 16) && aligned(queries, 16), "base/queries must be 16-byte aligned");
    ANN_REQUIRE(ws_bytes >= make_labels_ws(nq, M, kt), "workspace too small");
    if (nq == 0) return ANN_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    int32_t *ent = cv.take<int32_t>((size_t)nq);
    int32_t *kk = cv.take<int32_t>((size_t)nq);
    int32_t *LL = cv.take<int32_t>((size_t)nq);
    int32_t *ids = cv.take<int32_t>((size_t)nq * kt);
    float *dist = cv.take<float>((size_t)nq * kt);
    int32_t *stats = cv.take<int32_t>((size_t)nq * 4);
    int32_t *tab = cv.take<int32_t>((size_t)nq * M);
    uint32_t *counter = cv.take<uint32_t>(64);
    int32_t *fl = cv.take<int32_t>((size_t)nq);
    int32_t *redo = cv.take<int32_t>((size_t)nq);
    if (table) tab = table;
    if (flags) fl = flags;
    const int nb = blocks_for(nq);
    hipLaunchKernelGGL(fill_value_kernel, dim3(blocks_for((int64_t)nq * M)), dim3(256), 0, st, tab,
                       (int64_t)nq * M, -1);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(fill_value_kernel, dim3(nb), dim3(256), 0, st, fl, (int64_t)nq, 0);
    ANN_LAUNCHED();
    // costs are distance counts, so the filter must not forget ids: 32-bit
    // ids in 2^13 slots; the rare query that overflows them (a probe chain
    // longer than the table allows) is searched again with 2^14 slots
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            hipLaunchKernelGGL(redo_mark_kernel, dim3(nb), dim3(256), 0, st, fl, nq, M, tab, redo);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(fill_value_kernel, dim3(1), dim3(64), 0, st,
                               reinterpret_cast<int32_t *>(counter), (int64_t)1, 0);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(count_kernel, dim3(nb), dim3(256), 0, st, redo, nq,
                               reinterpret_cast<int32_t *>(counter));
            ANN_LAUNCHED();
            int32_t nredo = 0;
            ANN_HIP(hipMemcpyAsync(&nredo, counter, 4, hipMemcpyDeviceToHost, st));
            ANN_HIP(hipStreamSynchronize(st));
            if (nredo == 0) break;
        }
        for (int m = 0; m < M; ++m) {
            for (int li = 0; li < n_L; ++li) {
                const int Lv = L_ladder[li];
                if (pass == 0)
                    hipLaunchKernelGGL(gather_entries_kernel, dim3(nb), dim3(256), 0, st, cand_hubs,
                                       M, m, hub_ids, nq, ent, kk, LL, kt, Lv);
                else
                    hipLaunchKernelGGL(gather_redo_kernel, dim3(nb), dim3(256), 0, st, cand_hubs, M,
                                       m, hub_ids, redo, nq, ent, kk, LL, kt, Lv);
                ANN_LAUNCHED();
                ann_search_plan p{};
                ann_status s = ann_default_plan(n, dim, R, Lv, &p);
                if (s != ANN_OK) return s;
                p.filter = ANN_FILTER_ID32;
                p.visited_log2 = pass == 0 ? 13 : 14;
                s = search_launch(base, n, dim, graph, R, queries, nq, ent, 0, kk, LL, kt, ids,
                                  dist, stats, nullptr, 0, p, counter, st);
                if (s != ANN_OK) return s;
                hipLaunchKernelGGL(score_kernel, dim3(nb), dim3(256), 0, st, ids, stats, truth, kt,
                                   hits, nq, M, m, tab, fl);
                ANN_LAUNCHED();
            }
        }
    }
    hipLaunchKernelGGL(choose_kernel, dim3(nb), dim3(256), 0, st, tab, cand_hubs, nq, M, labels);
    ANN_LAUNCHED();
    return ANN_OK;
}
