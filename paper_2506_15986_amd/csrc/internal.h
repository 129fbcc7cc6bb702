// Internal cross-file declarations of libann (sizes of composite workspaces).
#pragma once

#include "common.h"

namespace ann {

struct Carve {
    unsigned char *p;
    template <typename T> T *take(size_t count)
    {
        T *r = reinterpret_cast<T *>(p);
        p += round_up(count * sizeof(T), 256);
        return r;
    }
};

size_t knn_workspace(int64_t n, int64_t rows, int dim, int K);
size_t build_graph_ws(int64_t n, int dim, int K, int R);
size_t medoid_ws(int64_t n, int dim);
size_t select_hubs_ws(int64_t n, int dim, int nh);
size_t hub_features_ws(int64_t n, int nh);
size_t make_labels_ws(int nq, int M, int kt);
size_t tower_forward_ws(int rows, const ann_tower *w);
size_t train_step_ws(int batch, int nh, int din_q, int din_h, int hidden, int dout);
ann_status search_launch(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                         int32_t R, const float *queries, int32_t nq, const int32_t *entry_ids,
                         int32_t medoid, const int32_t *k, const int32_t *L, int32_t k_max,
                         int32_t *out_ids, float *out_dist, int32_t *stats, int32_t *trace,
                         int32_t trace_cap, const ann_search_plan &p, uint32_t *counter,
                         hipStream_t st, bool widest_first = false);

// bytes of the search workspace: the work counter, and for a launch that
// orders its queries widest-expected-first, the order and its keys
size_t search_ws_bytes(int64_t nq);
ann_status validate_plan(const ann_search_plan &p);
size_t search_wave_lds(const ann_search_plan &p, int64_t n, int dim);
// host-side checks of ann_search's arguments; resolves a NULL plan to the
// default one in `p`.  Enqueues nothing.
ann_status search_check(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                        int32_t R, const float *queries, int32_t nq, const int32_t *entry_ids,
                        int32_t medoid, const int32_t *k, const int32_t *L, int32_t k_max,
                        int32_t *out_ids, float *out_dist, int32_t *trace, int32_t trace_cap,
                        const ann_search_plan *plan, void *workspace, size_t ws_bytes,
                        ann_search_plan &p);
// the entry stage's register-pool search over the hub graph (hubsearch.hip)
bool hub_search_supported(int n_hubs, int dim, int s, int L);
ann_status hub_search_launch(const float *emb, int n_hubs, int dim, const int32_t *graph, int s,
                             const float *qemb, int nq, int start, int L, int32_t *best,
                             float *best_d2, int32_t *stats, int32_t *trace, int trace_cap,
                             hipStream_t st);
ann_status tower_forward_run(const ann_tower &w, const float *x, const int32_t *idx, int rows,
                             float *out, void *ws, hipStream_t st);

}  // namespace ann
