/*
 * ann.h — C ABI of libann, the MI355X (gfx950) implementation of the GATE
 * query path: best-first beam search over a proximity graph (Algorithm 1),
 * entered at a query-aware hub chosen by a two-tower model through a
 * navigation graph over hub nodes (high-tier graph section).
 *
 * Conventions for every entry point
 *  - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *    allocates and owns every buffer (typically PyTorch tensors); the library
 *    never frees caller memory.  Opaque handles are the only library-owned
 *    objects and are released by the matching *_destroy call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls validate their arguments on the host, enqueue work on `stream` and
 *    return without synchronising, unless the comment says the call
 *    synchronises (calls that return host values do).
 *  - Scratch memory is caller-provided (`workspace`, `ws_bytes`); the size a
 *    call needs is returned by ann_workspace_size() for the same arguments.
 *  - On any status other than ANN_OK nothing has been enqueued and no output
 *    has been written, except where a comment says otherwise (device-side
 *    per-query checks are reported through per-query flags).
 *  - Nothing crosses the ABI except status codes: no exceptions, no exit(),
 *    no printing.  ann_last_error() returns the text of the last non-OK
 *    status raised on the calling thread.
 *  - Ordering convention: every "nearest" list is ordered by the key
 *    (squared L2 distance, id) — ties go to the smaller id.
 */
#ifndef ANN_H
#define ANN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ANN_OK = 0,
    ANN_EINVAL = 1,   /* bad argument (null, out of range, misaligned, ...) */
    ANN_ENOMEM = 2,   /* workspace too small */
    ANN_EDEVICE = 3,  /* HIP error; the HIP error text is in ann_last_error() */
    ANN_ENOTSUP = 4   /* valid but beyond the compiled kernel limits */
} ann_status;

/* Text of the last non-OK status on this thread ("" if none).  The pointer
 * stays valid until the next call on the same thread. */
const char *ann_last_error(void);

/* ABI version (major * 100 + minor). */
int32_t ann_version(void);

/* Operation codes for ann_workspace_size(). */
enum {
    ANN_OP_SEARCH = 1,
    ANN_OP_BUILD_GRAPH = 2,
    ANN_OP_GT_KNN = 3,
    ANN_OP_SELECT_HUBS = 4,
    ANN_OP_ENTRY_SELECT = 5,
    ANN_OP_MAKE_LABELS = 6,
    ANN_OP_HUB_FEATURES = 7,
    ANN_OP_TRAIN_STEP = 8
};

/* Bytes of workspace the operation needs.  Arguments per op:
 *   SEARCH        n, dim, p0 = nq,        p1 = unused
 *   BUILD_GRAPH   n, dim, p0 = knn_k,     p1 = R
 *   GT_KNN        n, dim, p0 = nq,        p1 = k
 *   SELECT_HUBS   n, dim, p0 = n_hubs,    p1 = unused
 *   ENTRY_SELECT  nq, dim, p0 = hidden,   p1 = embed dim
 *   MAKE_LABELS   n, dim, p0 = nq,        p1 = M (candidates per query)
 *   HUB_FEATURES  n, dim, p0 = n_hubs,    p1 = R
 *   TRAIN_STEP    batch, dim, p0 = n_hubs, p1 = hidden
 * Returns 0 for an unknown op. */
size_t ann_workspace_size(int32_t op, int64_t n, int32_t dim, int32_t p0, int32_t p1);

/* ------------------------------------------------------------------------ */
/* Beam search (Algorithm 1, read as the bounded-pool best-first search).    */

/* Launch plan: how one batched search launch maps onto the GPU.  Obtain
 * defaults from ann_default_plan() or tuned values from
 * ann_autotune_search(); all fields are plain values. */
typedef struct ann_search_plan {
    int32_t pool_cap;        /* largest beam width L the launch supports (<= 512) */
    int32_t visited_log2;    /* LDS visited table = 2^visited_log2 id slots (8..14) */
    int32_t group;           /* lanes that cooperate on one vector gather: 8 or 16 */
    int32_t waves_per_block; /* 1, 2 or 4 independent wavefronts per workgroup */
    int32_t blocks;          /* persistent grid size; 0 = as many as fit on the GPU */
    int32_t fp64;            /* 1 = FP64 distances (diagnostic mode), 0 = FP32 */
} ann_search_plan;

/* Fills *plan with the default plan for (n, dim, R, L_max).  host pointer. */
ann_status ann_default_plan(int64_t n, int32_t dim, int32_t R, int32_t L_max,
                            ann_search_plan *plan);

/* Batched best-first search.
 *   base      n x dim FP32 row-major, 16-byte aligned, dim % 4 == 0, dim <= 1024
 *   graph     n x R int32 neighbour ids, -1 = empty slot, 1 <= R <= 64
 *   queries   nq x dim FP32 row-major, 16-byte aligned
 *   entry_ids nq entry node ids, or NULL = `medoid` for every query
 *   k, L      nq int32 each: result count and beam width per query;
 *             1 <= k[i] <= L[i] <= plan->pool_cap and k[i] <= k_max
 *   out_ids   nq x k_max int32 (row i: the k[i] best ids, then -1)
 *   out_dist  nq x k_max FP32 squared L2 distances (then +inf)
 *   stats     nq x 4 int32 or NULL: [ndc_unique, ndc_exec, hops, flags];
 *             flags bit0 = the LDS visited table overflowed (results are still
 *             exact, ndc_unique may over-count), bit1 = invalid per-query
 *             arguments (k/L/entry out of range: the row is left -1/+inf)
 *   trace     nq x trace_cap int32 or NULL: ids expanded, in order, -1 padded
 *   plan      host pointer or NULL (= default plan for L_max = max over L is not
 *             known on the host, so NULL means pool_cap 256)
 *   workspace ann_workspace_size(ANN_OP_SEARCH, n, dim, nq, 0) bytes
 * With nq == 0 the per-query pointers may be NULL and nothing is enqueued.
 * Each query expands the best not-yet-expanded pool entry until none is left;
 * the FP32 (or FP64) distance of every newly seen neighbour is one distance
 * computation.  Ties are broken by the smaller id. */
ann_status ann_search(const float *base, int64_t n, int32_t dim,
                      const int32_t *graph, int32_t R,
                      const float *queries, int32_t nq,
                      const int32_t *entry_ids, int32_t medoid,
                      const int32_t *k, const int32_t *L, int32_t k_max,
                      int32_t *out_ids, float *out_dist, int32_t *stats,
                      int32_t *trace, int32_t trace_cap,
                      const ann_search_plan *plan,
                      void *workspace, size_t ws_bytes, void *stream);


/* ------------------------------------------------------------------------ */
/* Graph construction (the proximity graph G of Definition 1).              */

/* Exact k nearest neighbours of each query among the base vectors (the
 * ground truth of the recall of Eq. 1).  Rows ordered by (squared L2, id).
 *   base        n x dim FP32; queries nq x dim FP32
 *   exclude_self  nonzero: query i is base row i and id i is skipped
 *   out_ids     nq x k int32 (-1 padded when n < k), out_dist nq x k FP32
 *   workspace   ann_workspace_size(ANN_OP_GT_KNN, n, dim, nq, k) bytes
 * Data whose values are all integers in [0,255] with dim % 32 == 0 run on the
 * int8 matrix cores (exact); other data use FP64 distances (exact on data
 * held on a dyadic grid).  Synchronises `stream`. */
ann_status ann_gt_knn(const float *base, int64_t n, int32_t dim, const float *queries,
                      int32_t nq, int32_t k, int32_t exclude_self, int32_t *out_ids,
                      float *out_dist, void *workspace, size_t ws_bytes, void *stream);

/* The medoid (navigating node): the base point nearest the FP64 mean, by
 * (squared distance summed in dimension order, id).  *medoid is a host
 * pointer.  workspace: ann_workspace_size(ANN_OP_BUILD_GRAPH, n, dim, 1, 3)
 * is always enough.  Synchronises `stream`. */
ann_status ann_medoid(const float *base, int64_t n, int32_t dim, int32_t *medoid,
                      void *workspace, size_t ws_bytes, void *stream);

/* Proximity graph: exact kNN (knn_k, self excluded) -> alpha-RNG pruning to
 * at most R-2 neighbours (candidate c is dropped when a kept o has
 * alpha^2 d2(o,c) <= d2(p,c); alpha^2 is formed in FP64 from the FP32 alpha)
 * -> medoid -> connectivity repair: slot R-2 receives forward bridges (the
 * smallest unreached id, linked from its nearest reached node with that slot
 * free) and slot R-1 reverse bridges (the smallest id that cannot reach the
 * medoid, linked to its nearest node that can).  Afterwards every node is
 * reachable from the medoid and reaches it.
 *   graph    n x R int32 output, -1 padded
 *   medoid   host int32 output
 *   bridges  host int32[2] output (forward, reverse bridge counts) or NULL
 *   workspace ann_workspace_size(ANN_OP_BUILD_GRAPH, n, dim, knn_k, R)
 * Requires 3 <= R <= 64, R-2 <= knn_k < n, alpha >= 1.  Synchronises. */
ann_status ann_build_graph(const float *base, int64_t n, int32_t dim, int32_t knn_k, int32_t R,
                           float alpha, int32_t *graph, int32_t *medoid, int32_t *bridges,
                           void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Hub nodes and their topology features (hub extraction and feature         */
/* distillation sections).                                                   */

/* Hub nodes (Definition 3) on Lloyd k-means clusters.  init_ids (n_hubs
 * base ids, device) seed the centroids.  Each step assigns every point to
 * argmin_c (d2(x, mu_c), c) with d2 the FP64 sum over dimensions in order
 * without fused multiply-add, then sets mu_c to the FP64 mean of its members
 * (an empty cluster keeps its centroid); the loop stops after a step that
 * changes no assignment or after `iters` steps.  hub_ids[c] is the member of
 * cluster c nearest mu_c by (d2, id); an empty cluster takes the nearest
 * point that is not yet a hub, in cluster order.
 *   centroids  n_hubs x dim FP64 output or NULL; assign n int32 output or NULL
 *   steps      host int32 output (assignment steps run) or NULL
 *   workspace  ann_workspace_size(ANN_OP_SELECT_HUBS, n, dim, n_hubs, 0)
 * Synchronises `stream`. */
ann_status ann_select_hubs(const float *base, int64_t n, int32_t dim, int32_t n_hubs,
                           int32_t iters, const int32_t *init_ids, int32_t *hub_ids,
                           double *centroids, int32_t *assign, int32_t *steps,
                           void *workspace, size_t ws_bytes, void *stream);

/* 32 topology features per hub, standardised per column across hubs
 * (population std; a constant column becomes 0) unless standardise == 0.
 * A guided walk of at most h hops and wcap nodes samples, at each node u,
 * the ceil(x/2) nearest and floor(x/2) farthest neighbours with
 * x = max(2, ceil(MinDeg * deg(u) / MaxDeg)).  With nu the mean distance of
 * a node to its first neighbour slot, the columns are:
 *   0 out-degree / R            1 in-degree / mean in-degree
 *   2-6 log2(1 + walk nodes first reached at hop 1..5)
 *   7 log2(1 + sampled walk edges)
 *   8-11 mean, min, max, std of dist(hub, out-neighbour) / nu
 *   12-15 the same over the walk nodes
 *   16 cluster size / (n / n_hubs)   17 dist(hub, centroid) / nu
 *   18 dist(hub, medoid) / nu        19 share of walk nodes in other clusters
 *   20 mean out-degree / R and 21 mean in-degree / mean in-degree of walk nodes
 *   22 mean sampled-edge length / nu  23 deepest walk hop / h   24-31 zero
 *   assign     n int32 cluster of each point; centroids n_hubs x dim FP64
 *   features   n_hubs x 32 FP32 output; walk_sizes n_hubs x 6 int32 or NULL
 *              (walk nodes per hop 0..5)
 *   workspace  ann_workspace_size(ANN_OP_HUB_FEATURES, n, dim, n_hubs, R) */
ann_status ann_hub_features(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                            int32_t R, int32_t medoid, const int32_t *hub_ids, int32_t n_hubs,
                            const int32_t *assign, const double *centroids, int32_t h,
                            int32_t wcap, int32_t standardise, float *features,
                            int32_t *walk_sizes, void *workspace, size_t ws_bytes,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ANN_H */
