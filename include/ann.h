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

/* *result (host) = max |x_i| over x[0..count).  workspace >= 4 bytes.
 * Synchronises `stream`. */
ann_status ann_max_abs(const float *x, int64_t count, float *result, void *workspace,
                       size_t ws_bytes, void *stream);

/* Operation codes for ann_workspace_size(). */
enum {
    ANN_OP_SEARCH = 1,
    ANN_OP_BUILD_GRAPH = 2,
    ANN_OP_GT_KNN = 3,
    ANN_OP_SELECT_HUBS = 4,
    ANN_OP_ENTRY_SELECT = 5,
    ANN_OP_MAKE_LABELS = 6,
    ANN_OP_HUB_FEATURES = 7
};

/* Bytes of workspace the operation needs.  Arguments per op:
 *   SEARCH        n, dim, p0 = nq,        p1 = unused
 *   BUILD_GRAPH   n, dim, p0 = knn_k,     p1 = R
 *   GT_KNN        n, dim, p0 = nq,        p1 = k
 *   SELECT_HUBS   n, dim, p0 = n_hubs,    p1 = unused
 *   ENTRY_SELECT  nq, dim, p0 = hidden,   p1 = embed dim
 *   MAKE_LABELS   n, dim, p0 = nq,        p1 = M (candidates per query)
 *   HUB_FEATURES  n, dim, p0 = n_hubs,    p1 = R
 * Returns 0 for an unknown op.  The tower, training and entry-selection
 * calls have their own size functions below. */
size_t ann_workspace_size(int32_t op, int64_t n, int32_t dim, int32_t p0, int32_t p1);

/* ------------------------------------------------------------------------ */
/* Beam search (Algorithm 1, read as the bounded-pool best-first search).    */

/* Launch plan: how one batched search launch maps onto the GPU.  Obtain
 * defaults from ann_default_plan() or tuned values from
 * ann_autotune_search(); all fields are plain values. */
typedef struct ann_search_plan {
    int32_t pool_cap;        /* largest beam width L the launch supports (<= 1024) */
    int32_t visited_log2;    /* LDS visited filter = 2^visited_log2 slots (8..14) */
    int32_t group;           /* lanes that cooperate on one vector gather: 4 (dim <= 64), 8 (dim <= 128) or 16 */
    int32_t waves_per_block; /* 1, 2 or 4 independent wavefronts per workgroup */
    int32_t blocks;          /* persistent grid size; 0 = as many as fit on the GPU */
    int32_t fp64;            /* 1 = FP64 distances (diagnostic mode), 0 = FP32 */
    int32_t filter;          /* visited filter form, one of ANN_FILTER_* */
    int32_t waves_per_query; /* wavefronts that share one query: 1 (0 = 1), or 2 / 4 (FP32, group 16;
                                the workgroup is then one query's waves, so
                                waves_per_block must equal waves_per_query) */
    int32_t query_order;     /* ANN_ORDER_WIDEST_FIRST (0) or ANN_ORDER_AS_GIVEN (1), see ann_search */
} ann_search_plan;

/* Order in which a search launch takes its queries (results are the same in
 * any order; only the launch's duration depends on it). */
enum { ANN_ORDER_WIDEST_FIRST = 0, ANN_ORDER_AS_GIVEN = 1 };

/* Visited filter forms (per wavefront, in LDS).  Every form answers "seen"
 * only for ids it was given; the hash forms may forget an id, which costs a
 * repeated distance computation but never changes the results.
 *   AUTO   BITSET when n bits fit in the TAG16 table's bytes, else TAG12 when
 *          its tags fit in 11 bits, else TAG16 when they fit in 15, else ID32
 *   BITSET one bit per id (exact); needs ceil(n/32) <= 2^visited_log2 words
 *   TAG16  4-way set-associative table of 16-bit tags, 2 bytes per slot; an
 *          invertible hash makes (set, tag) name one id; needs
 *          ceil(log2 n) - (visited_log2 - 2) <= 15
 *   ID32   linear-probing table of 32-bit ids, 4 bytes per slot
 *   TAG12  as TAG16 with five 12-bit ways per 64-bit set in the same bytes
 *          (2^visited_log2 / 4 sets, 5 slots each); needs
 *          ceil(log2 n) - (visited_log2 - 2) <= 11 */
enum { ANN_FILTER_AUTO = 0, ANN_FILTER_BITSET = 1, ANN_FILTER_TAG16 = 2, ANN_FILTER_ID32 = 3,
       ANN_FILTER_TAG12 = 4 };

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
 * With plan->query_order == ANN_ORDER_WIDEST_FIRST (the default) queries are
 * taken widest-expected-first: a pre-pass orders them by L[i] times the FP32
 * squared distance from query i to its entry, largest first (the order lives
 * in the workspace), so that the longest searches do not start last.  With
 * ANN_ORDER_AS_GIVEN they are taken in index order (for pipelines that keep
 * several launches in flight, where the next launch fills the tail).  Every
 * query's results are the same in any order.
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


/* ann_search without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and errors are those of ann_search;
 * the scratch that ann_search takes from `workspace` (the persistent
 * launch's work counter, and the widest-first query order with its keys)
 * lives instead in a fixed array inside this library: 256 bytes + 8 bytes per
 * query for up to ANN_NOALLOC_MAX_QUERIES queries (about 8 MiB), one copy
 * per GPU, resolved on the first call on each device and held until the
 * process ends.  The call allocates nothing (no hipMalloc, no allocating
 * library routine).  nq above ANN_NOALLOC_MAX_QUERIES returns ANN_EINVAL.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (the counter is cleared by a kernel at the start of each call):
 * calls that overlap on one GPU (on different streams, or from different
 * threads) race and give undefined results; serialise them on one stream. */
enum { ANN_NOALLOC_MAX_QUERIES = 1 << 20 };

ann_status ann_search_noalloc(const float *base, int64_t n, int32_t dim,
                              const int32_t *graph, int32_t R,
                              const float *queries, int32_t nq,
                              const int32_t *entry_ids, int32_t medoid,
                              const int32_t *k, const int32_t *L, int32_t k_max,
                              int32_t *out_ids, float *out_dist, int32_t *stats,
                              int32_t *trace, int32_t trace_cap,
                              const ann_search_plan *plan, void *stream);

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

/* The same pipeline with candidate lists drawn from overlapping groups, for
 * indexes too large for an all-pairs kNN (not a step of the paper, which
 * assumes a built proximity graph: a construction shortcut for the 10M-point
 * workload).  groups is n x n_member int32 (device): row i lists the groups
 * of point i, column 0 its home group in [0, n_groups), further columns
 * other groups or -1 (a repeated label counts once).  The candidates of
 * point i are the exact knn_k nearest, by (squared L2, id), among the points
 * whose row lists i's home group, i excluded; fewer (then -1 / +inf padded)
 * when that set is smaller.  Then ann_graph_from_candidates.  Cost: the sum
 * over groups of (home points x members).  The labels are read on the host
 * (the call synchronises).
 *   workspace  ann_build_graph_partitioned_workspace_size(n, dim, knn_k, R,
 *              largest member set, largest home set) bytes
 * Errors: EINVAL for a home label outside [0, n_groups), another label
 * outside [-1, n_groups), n_member < 1, or a workspace that is too small. */
size_t ann_build_graph_partitioned_workspace_size(int64_t n, int32_t dim, int32_t knn_k, int32_t R,
                                                  int64_t max_members, int64_t max_home);

ann_status ann_build_graph_partitioned(const float *base, int64_t n, int32_t dim, int32_t knn_k,
                                       int32_t R, float alpha, const int32_t *groups,
                                       int32_t n_member, int32_t n_groups, int32_t *graph,
                                       int32_t *medoid, int32_t *bridges, void *workspace,
                                       size_t ws_bytes, void *stream);

/* The first step of ann_build_graph_partitioned for the home points of
 * groups [g_begin, g_end) only, so that a caller can split the work:
 * writes their rows of cand (n x knn_k int32, device) and cand_d2 (n x knn_k
 * float64 squared distances, device); other rows are left untouched.
 *   workspace  ann_group_candidates_workspace_size(dim, knn_k, largest
 *              member set, largest home set) bytes (over all groups)
 * Errors as ann_build_graph_partitioned, and EINVAL unless
 * 0 <= g_begin <= g_end <= n_groups.  Synchronises. */
size_t ann_group_candidates_workspace_size(int32_t dim, int32_t knn_k, int64_t max_members,
                                           int64_t max_home);

ann_status ann_group_candidates(const float *base, int64_t n, int32_t dim, int32_t knn_k,
                                const int32_t *groups, int32_t n_member, int32_t n_groups,
                                int32_t g_begin, int32_t g_end, int32_t *cand, double *cand_d2,
                                void *workspace, size_t ws_bytes, void *stream);

/* Graph from given candidate lists (rows sorted by (squared L2, id), -1 /
 * +inf padded; cand_d2 the FP64 squared distances): alpha pruning, the
 * medoid and the connectivity repair of ann_build_graph.  A repair bridge is
 * the first eligible entry of the unreached point's list when there is one,
 * else the argmin over all eligible points; for the exact global kNN lists
 * of ann_build_graph the two rules pick the same node.
 *   workspace  ann_graph_from_candidates_workspace_size(n, dim, R) bytes
 * Requires 3 <= R <= 64, R-2 <= knn_k <= 1024, alpha >= 1.  Synchronises. */
size_t ann_graph_from_candidates_workspace_size(int64_t n, int32_t dim, int32_t R);

ann_status ann_graph_from_candidates(const float *base, int64_t n, int32_t dim,
                                     const int32_t *cand, const double *cand_d2, int32_t knn_k,
                                     int32_t R, float alpha, int32_t *graph, int32_t *medoid,
                                     int32_t *bridges, void *workspace, size_t ws_bytes,
                                     void *stream);

/* Candidate lists of an NSG-style graph (the base index the paper builds on,
 * whose candidates come from a search for each point plus its nearest
 * neighbours): row i of the output is the union of row i of a_ids
 * (n x a_w int32, device; e.g. the pool of a search for base point i) and
 * row i of b_ids (n x b_w int32, device; e.g. its exact kNN list), with -1
 * entries, i itself and repeats dropped, ordered by (FP64 squared L2 to
 * base point i, id), then -1 / +inf padded to a_w + b_w.  The distances are
 * recomputed here (eight partial sums over dimensions j mod 8, combined
 * pairwise; exact on data held on a dyadic grid), so the input lists carry
 * ids only.  The result feeds ann_graph_from_candidates with
 * knn_k = a_w + b_w and alpha = 1 (NSG's MRNG rule).
 *   out_ids   n x (a_w + b_w) int32 (device), out_d2 the same shape FP64
 *   workspace ann_merge_candidates_workspace_size() bytes (an error flag)
 * Errors: EINVAL unless 1 <= a_w + b_w <= 1024, or when an input id lies
 * outside [-1, n) (such an id counts as absent in the output, which is
 * still written).  Synchronises `stream`. */
size_t ann_merge_candidates_workspace_size(void);

ann_status ann_merge_candidates(const float *base, int64_t n, int32_t dim, const int32_t *a_ids,
                                int32_t a_w, const int32_t *b_ids, int32_t b_w, int32_t *out_ids,
                                double *out_d2, void *workspace, size_t ws_bytes, void *stream);

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

/* Seeded start for ann_select_hubs (the paper leaves the k-means start
 * open): n_hubs distinct base ids written to the HOST array ids, drawn by
 * Floyd's sampling (for j = n - n_hubs .. n - 1 draw t in [0, j], take t or,
 * if t is taken, j; ids in the order taken) with the i-th draw
 * t = floor(x_i (j + 1) / 2^64), x_i the i-th SplitMix64 output from state
 * `seed`.  Host-only; EINVAL unless 1 <= n_hubs <= n < 2^31. */
ann_status ann_hub_init_ids(int64_t n, int32_t n_hubs, uint64_t seed, int32_t *ids);

/* Hub nodes (Definition 3) on hierarchical balanced k-means clusters
 * (Algorithm 2): levels rounds split every cluster into k children, giving
 * n_c = k^levels clusters (cluster p*k + j of a round is child j of cluster p
 * of the round before).  A split runs `iters` passes over the parent's
 * members in id order; each pass starts from empty children and puts each
 * member into the child j of smallest d2(x, mu_j) + lambda * (2 (s_j - m/k)
 * + 1), where s_j is the size child j has reached so far in the pass and m
 * the parent's size: the change in the balance objective of Definition 2
 * when x joins child j (the printed size term read as that change; the other
 * children's terms are common to every j).  Ties go to the smaller j; d2 and
 * the penalty are FP64 without fused multiply-add.  After each pass mu_j is
 * the FP64 mean of its members (an empty child keeps its centroid).  Child j
 * starts at the parent's member at position floor((2j + 1) m / (2k)) (a
 * parent without members passes its centroid on).  Hubs as ann_select_hubs.
 *   k          2..64; k^levels <= min(n, 2^20)
 *   lambda     >= 0 (0: hierarchical k-means without the size term)
 *   hub_ids    n_c int32 output; centroids n_c x dim FP64 output or NULL;
 *   assign     n int32 output (final cluster of every point)
 *   workspace  ann_select_hubs_hbkm_workspace_size(n, dim, k, levels) bytes
 * Synchronises `stream`. */
size_t ann_select_hubs_hbkm_workspace_size(int64_t n, int32_t dim, int32_t k, int32_t levels);

ann_status ann_select_hubs_hbkm(const float *base, int64_t n, int32_t dim, int32_t k,
                                int32_t levels, double lambda, int32_t iters, int32_t *hub_ids,
                                double *centroids, int32_t *assign, void *workspace,
                                size_t ws_bytes, void *stream);

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

/* ------------------------------------------------------------------------ */
/* Two-tower entry model (two-tower score of the preliminaries; projection   */
/* network and contrastive loss of the high-tier graph section).             */
/*   tower(x) = normalise(W2 . relu(W1 . x + b1) + b2)                        */
/* FP32 master weights with BF16 working copies; every matrix product takes  */
/* BF16 operands (round to nearest even) and accumulates in FP32 on the      */
/* matrix cores.  Rounded operands: the tower input, the weights, the hidden  */
/* activation after ReLU and, backwards, the pre-activation gradients that   */
/* enter the weight and input products.  Bias, ReLU, normalisation, logits   */
/* and softmax stay in FP32.  Every reduction runs in a fixed order.         */

typedef struct ann_tower {
    int32_t din, hidden, dout;
    float in_scale; /* the input is multiplied by in_scale before the BF16 rounding
                       (a power of two keeps it exact) */
    float *W1;      /* hidden x din, FP32 master */
    float *b1;      /* hidden */
    float *W2;      /* dout x hidden */
    float *b2;      /* dout */
    uint16_t *W1b;  /* BF16 copy of W1 (bit patterns) */
    uint16_t *W2b;  /* BF16 copy of W2 */
} ann_tower;

typedef struct ann_tower_grads {
    float *gW1, *gb1, *gW2, *gb2;   /* same shapes as the parameters */
} ann_tower_grads;

typedef struct ann_adam_state {
    float *mW1, *vW1, *mb1, *vb1, *mW2, *vW2, *mb2, *vb2;   /* zero-initialised */
} ann_adam_state;

/* Hub tower input: row c = [ base row hub_ids[c] * vec_scale | features row c ]
 * (n_hubs x (dim + n_feat) FP32).  n_feat may be 0 (the hub vectors alone). */
ann_status ann_hub_input(const float *base, int64_t n, int32_t dim, const int32_t *hub_ids,
                         int32_t n_hubs, const float *features, int32_t n_feat, float vec_scale,
                         float *out, void *stream);

/* Refreshes the BF16 copies from the FP32 masters (RNE). */
ann_status ann_tower_sync(const ann_tower *tower, void *stream);

size_t ann_tower_workspace_size(const ann_tower *tower, int32_t rows);

/* Unit embeddings of `rows` FP32 input rows (rows x din) -> out (rows x dout). */
ann_status ann_tower_forward(const ann_tower *tower, const float *x, int32_t rows, float *out,
                             void *workspace, size_t ws_bytes, void *stream);

size_t ann_train_workspace_size(int32_t batch, int32_t n_hubs, int32_t din_q, int32_t din_h,
                                int32_t hidden, int32_t dout);

/* One contrastive training step (the loss of Eq. 2 / Eq. 4 taken
 * query-anchored over all hubs, positive inside the denominator):
 *   L = mean_i [ logsumexp_h(s_ih) - s_i,y_i ],  s_ih = <e_q_i, e_h> / tau
 * with e_q = query tower of train_q[batch_idx[i]] and e_h = hub tower of
 * hub_in (n_hubs x din_h: hub vector then its features), y_i =
 * labels[batch_idx[i]].  Writes gradients into qg / hg, the mean loss to
 * *loss (device FP32), the embeddings to q_emb / h_emb when non-NULL, and
 * when step >= 1 applies Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * correction with t = step) to both towers and refreshes their BF16 copies.
 * step == 0 computes gradients only.  hub_in_grad (n_hubs x din_h, device,
 * or NULL) receives dL/d hub_in (the input's BF16 rounding taken as the
 * identity), for an upstream module such as the fusion embedding. */
ann_status ann_train_step(ann_tower *query_tower, ann_tower *hub_tower,
                          const ann_tower_grads *qg, const ann_tower_grads *hg,
                          const ann_adam_state *qa, const ann_adam_state *ha,
                          const float *train_q, const int32_t *batch_idx, int32_t batch,
                          const int32_t *labels, const float *hub_in, int32_t n_hubs,
                          float tau, float lr, int32_t step, float *loss, float *q_emb,
                          float *h_emb, float *hub_in_grad, void *workspace, size_t ws_bytes,
                          void *stream);

size_t ann_train_hub_workspace_size(int32_t hubs, int32_t P, int32_t N, int32_t din_q,
                                    int32_t din_h, int32_t hidden, int32_t dout);

/* One training step of Eq. 4 read hub-anchored over each hub's positive and
 * negative queues (Definition 4): the batch holds `hubs` hubs (rows
 * hub_idx[i] of hub_in) and hubs x (P + N) queries (rows q_idx[...] of
 * train_q), hub i owning q_idx[i*(P+N) .. i*(P+N)+P-1] as positives and the
 * next N as negatives.  With s_iq = <e_h_i, e_q> / tau and LSE_i over hub i's
 * P + N scores:
 *   L = mean_i [ P * LSE_i - sum_{q positive for i} s_iq ]
 * (the printed per-hub sum of -log softmax over the positives).  Gradients,
 * loss, embeddings and Adam as ann_train_step.  P >= 1, N >= 0. */
ann_status ann_train_step_hub(ann_tower *query_tower, ann_tower *hub_tower,
                              const ann_tower_grads *query_grads, const ann_tower_grads *hub_grads,
                              const ann_adam_state *query_adam, const ann_adam_state *hub_adam,
                              const float *train_q, const int32_t *q_idx, const int32_t *hub_idx,
                              int32_t hubs, int32_t P, int32_t N, const float *hub_in, float tau,
                              float lr, int32_t step, float *loss, float *q_emb, float *h_emb,
                              void *workspace, size_t ws_bytes, void *stream);

/* Fusion embedding augmentation (Eq. 3): multi-head attention of each hub's
 * vector p (dp values) over its S topology tokens U (du values each, masked
 * slots absent):
 *   q = p WQ^T, K_s = U_s WK^T, V_s = U_s WV^T   (heads x dk channels; head j
 *                                                 owns channels j*dk .. j*dk+dk-1)
 *   a_j = softmax over present s of <q_j, K_s,j> / sqrt(dk)
 *   F = concat_j( sum_s a_j,s V_s,j ) WO^T         (df values)
 * A hub without present tokens gets F = 0.  FP32, fixed summation order.
 * Limits: heads <= 16, heads * dk <= 64, df <= 64, S <= 64. */
typedef struct ann_fusion {
    int32_t heads, dk, dp, du, df;
    float *WQ;   /* heads*dk x dp */
    float *WK;   /* heads*dk x du */
    float *WV;   /* heads*dk x du */
    float *WO;   /* df x heads*dk */
} ann_fusion;

/* The fusion embedding's inputs for each hub (Eq. 3 with the topology tokens
 * read as the relative positions of the hub's graph neighbours): p row c =
 * base row hub_ids[c] * scale (n_hubs x dim), U[c][s] = (base row w - base row
 * hub_ids[c]) * scale for the neighbour w in graph slot s of the hub
 * (n_hubs x R x dim; zeros for an empty slot), mask[c][s] = 1 when slot s
 * holds a neighbour (n_hubs x R uint8).  FP32 (subtract, then multiply by
 * scale, a power of two in practice).  Enqueues only; ids are not checked on
 * the device (the hub ids and graph must lie in [0, n), -1 for empty slots). */
ann_status ann_fusion_tokens(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                             int32_t R, const int32_t *hub_ids, int32_t n_hubs, float scale,
                             float *p, float *U, uint8_t *mask, void *stream);

/* F (n_hubs x df) from p (n_hubs x dp), U (n_hubs x S x du) and mask
 * (n_hubs x S, 1 = present); all device.  Enqueues only. */
ann_status ann_fusion_forward(const ann_fusion *f, const float *p, const float *U,
                              const uint8_t *mask, int32_t n_hubs, int32_t S, float *F,
                              void *stream);

size_t ann_fusion_workspace_size(const ann_fusion *f, int32_t n_hubs);

/* Gradients of the four matrices (same shapes, overwritten) given dL/dF
 * (n_hubs x df): per-hub partial gradients summed in hub order. */
ann_status ann_fusion_backward(const ann_fusion *f, const float *p, const float *U,
                               const uint8_t *mask, int32_t n_hubs, int32_t S, const float *dF,
                               float *gWQ, float *gWK, float *gWV, float *gWO, void *workspace,
                               size_t ws_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction with t =
 * step >= 1) on `count` FP32 parameters with their moment buffers. */
ann_status ann_adam_step(float *param, const float *grad, float *m, float *v, int64_t count,
                         float lr, int32_t step, void *stream);

/* Hop counts of Definition 4: out[q * n_hubs + h] (uint8, device) = the
 * length of the shortest path along the graph's edges from hub_ids[h] to
 * targets[q] (the query's nearest neighbour), 255 when unreachable or more
 * than 254 hops away.  Breadth-first search from 64 hubs at a time (one bit
 * per hub in a 64-bit word per node).  Hub and target ids are checked on the
 * host (EINVAL when out of range).
 *   workspace  ann_hop_table_workspace_size(n) bytes.  Synchronises. */
size_t ann_hop_table_workspace_size(int64_t n);

ann_status ann_hop_table(const int32_t *graph, int64_t n, int32_t R, const int32_t *hub_ids,
                         int32_t n_hubs, const int32_t *targets, int64_t nq, uint8_t *out,
                         void *workspace, size_t ws_bytes, void *stream);

/* Positive and negative query queues of Definition 4 from a hop table
 * (hops: nq x n_hubs uint8, device, as ann_hop_table writes it, 255 =
 * unreachable).  With m_h the smallest hop count of hub h over all queries,
 * query q is a positive of h when H(q, h) <= m_h + t_pos and a negative when
 * H(q, h) == 255 or H(q, h) >= m_h + t_neg (the definition's negatives,
 * "defined analogously", read with t_neg); a hub that reaches no query has
 * neither.  Queue h lists its query indices in increasing order; the queues
 * are concatenated hub after hub:
 *   pos_off, neg_off  n_hubs + 1 int64 (device): queue h spans
 *                     [off[h], off[h + 1]) of pos_q / neg_q
 *   pos_q, neg_q      int32 (device) with room for pos_cap / neg_cap entries
 *                     (NULL allowed with capacity 0)
 *   totals            host int64[2]: the two queues' total lengths
 * The call computes the offsets, copies the totals to the host
 * (synchronising `stream`), and fills the lists when they fit; when a
 * capacity is too small it returns ANN_ENOMEM after writing only the
 * offsets and totals, so a caller can size the lists and call again.
 *   workspace  ann_make_queues_workspace_size(nq, n_hubs) bytes
 * Requires 1 <= nq < 2^31, 1 <= n_hubs <= 2^20, t_pos, t_neg >= 0. */
size_t ann_make_queues_workspace_size(int64_t nq, int32_t n_hubs);

ann_status ann_make_queues(const uint8_t *hops, int64_t nq, int32_t n_hubs, int32_t t_pos,
                           int32_t t_neg, int64_t *pos_off, int64_t *neg_off, int32_t *pos_q,
                           int64_t pos_cap, int32_t *neg_q, int64_t neg_cap, int64_t *totals,
                           void *workspace, size_t ws_bytes, void *stream);

/* Navigation graph over hubs.  Rows of hub_emb are unit vectors, so
 * |e_i - e_j|^2 = 2 - 2 cos(e_i, e_j) and the order by squared L2 distance is
 * the cosine order: row i = the s hubs j != i of largest cosine with hub i,
 * found as the exact nearest neighbours by (FP64 squared L2, j).
 * *hub_entry (host) = the medoid of the embeddings, which is the hub of
 * largest cosine with their mean direction; the hub-graph search starts there.
 * workspace: ann_navgraph_workspace_size(n_hubs, dim, s).  Synchronises. */
size_t ann_navgraph_workspace_size(int32_t n_hubs, int32_t dim, int32_t s);

ann_status ann_navgraph_build(const float *hub_emb, int32_t n_hubs, int32_t dim, int32_t s,
                              int32_t *hub_graph, int32_t *hub_entry, void *workspace,
                              size_t ws_bytes, void *stream);

/* The entry stage's best-first search over the hub navigation graph (the
 * high-tier graph section's Algorithm 1 on the hub graph): for each query
 * embedding, the search of ann_search with k = 1, beam width L and an exact
 * visited set, from hub `start`, over unit hub embeddings by squared L2
 * (cosine order), specialised for small hub graphs: the pool lives in the
 * wavefront's registers, so L <= 64.
 *   emb        n_hubs x dim FP32 (16-byte aligned), dim % 4 == 0, 4 <= dim <= 256
 *   graph      n_hubs x s int32 hub indices, -1 = empty slot; 1 <= s <= 64
 *   qemb       nq x dim FP32 query embeddings (16-byte aligned)
 *   best       nq int32: the best hub; best_d2 nq FP32: its squared distance
 *   stats      nq x 2 int32 or NULL: distance computations, expansions
 *   trace      nq x trace_cap int32 or NULL: hubs expanded, in order, -1 padded
 * Requires 1 <= n_hubs <= 65536, 1 <= L <= 64, 0 <= start < n_hubs (else
 * ANN_ENOTSUP / ANN_EINVAL).  Enqueues only.  ann_entry_select uses it when
 * the model's shapes allow, the base search kernel otherwise. */
ann_status ann_hub_search(const float *emb, int32_t n_hubs, int32_t dim, const int32_t *graph,
                          int32_t s, const float *qemb, int32_t nq, int32_t start, int32_t L,
                          int32_t *best, float *best_d2, int32_t *stats, int32_t *trace,
                          int32_t trace_cap, void *stream);

typedef struct ann_entry_model {
    ann_tower query_tower;      /* BF16 copies must be current */
    const float *hub_emb;       /* n_hubs x query_tower.dout, unit rows */
    const int32_t *hub_graph;   /* n_hubs x s */
    int32_t n_hubs, s;
    const int32_t *hub_ids;     /* base id of each hub */
    int32_t hub_entry;          /* hub index where the hub-graph search starts */
    int32_t medoid;             /* fallback entry point */
    int32_t L_h;                /* beam width on the hub graph (<= 512) */
    float theta;                /* best cosine below theta -> medoid */
    ann_search_plan hub_plan;   /* plan of the hub-graph search; pool_cap 0 = the default
                                   plan for (n_hubs, embed dim, s, L_h) */
} ann_entry_model;

/* The model as a handle: ann_entry_model_create checks the fields of *desc
 * (the checks of ann_entry_select that need no queries and no device) and
 * returns in *out a host copy of it, to pass wherever a model is taken.  The
 * device pointers in it are borrowed: the caller keeps them alive and owns
 * them.  ann_entry_model_destroy frees the copy only (NULL is a no-op).
 * On a non-OK status *out is NULL. */
ann_status ann_entry_model_create(const ann_entry_model *desc, ann_entry_model **out);
void ann_entry_model_destroy(ann_entry_model *model);

size_t ann_entry_workspace_size(const ann_entry_model *model, int32_t nq);

/* Query-aware entry points: the query tower embeds each query; a best-first
 * search over the hub graph (k = 1 and beam width L_h, squared L2 between unit
 * embeddings, i.e. cosine order: ann_hub_search when L_h <= 64 and the hub
 * table fits its limits, else the ann_search kernel with model->hub_plan)
 * starts at model->hub_entry and returns the best hub h with cos = 1 - d2 / 2;
 * entry_ids[i] = hub_ids[h], or the medoid when cos < theta.  entry_score
 * (FP32 cosine) and best_hub may be NULL. */
ann_status ann_entry_select(const ann_entry_model *model, const float *queries, int32_t nq,
                            int32_t dim, int32_t *entry_ids, float *entry_score,
                            int32_t *best_hub, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Training labels for the entry model.  This takes the place of the paper's */
/* hop-count positive and negative queues (Definition 4) with the same       */
/* intent: which hub serves a query best.  For historical query i and each    */
/* candidate hub m (cand_hubs row i, nearest first), the batched beam search  */
/* (as ann_search) runs from that hub with each width of L_ladder (host,     */
/* increasing, kt <= L <= 512); the cost of (i, m) is the distance count      */
/* (ndc_unique) of the first width whose top-kt holds at least `hits` of the  */
/* query's true top-kt (truth row i).  The label is the candidate of least    */
/* cost, ties to the smaller hub index, or the first candidate when none      */
/* reaches the target.                                                        */
/*   table  nq x M int32 or NULL: the cost, -1 when no width reached it        */
/*   flags  nq int32 or NULL: bit0 = a search of that query overflowed the    */
/*          LDS visited table (its counts may include repeated nodes)         */
/*   workspace  ann_labels_workspace_size(nq, M, kt) bytes.  kt <= 64.        */
size_t ann_labels_workspace_size(int32_t nq, int32_t M, int32_t kt);

ann_status ann_make_labels(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                           int32_t R, const float *queries, int32_t nq, const int32_t *truth,
                           int32_t kt, int32_t hits, const int32_t *cand_hubs, int32_t M,
                           const int32_t *hub_ids, const int32_t *L_ladder, int32_t n_L,
                           int32_t *labels, int32_t *table, int32_t *flags, void *workspace,
                           size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batch driver: plan tuning, one-call query batches and HIP graphs.         */
/* Thousands of queries with uneven k and L run in one persistent search     */
/* launch; the plan (gather width, LDS filter size and form, waves per       */
/* workgroup) is chosen by timing candidates on a sample batch.              */

/* LDS bytes one wavefront of `plan` needs for n ids of dimension dim
 * (host-only, no GPU work); 0 when the plan's filter form cannot hold n ids. */
size_t ann_search_plan_lds(const ann_search_plan *plan, int64_t n, int32_t dim);

/* Candidate plans for (n, dim, R, L_max): writes up to `cap` plans to the
 * host array `plans` and returns how many there are (call with cap = 0 to
 * count).  pool_cap is L_max rounded up to 16; the candidates vary the
 * gather group, the filter size (visited_log2 10..13, form AUTO), the waves
 * per workgroup and, for group 16, the wavefronts per query (2, 4).
 * Host-only. */
int32_t ann_autotune_candidates(int64_t n, int32_t dim, int32_t R, int32_t L_max,
                                ann_search_plan *plans, int32_t cap);

/* Times each of the n_cand plans (host array) on the given batch — one
 * warm-up launch, then `reps` timed launches each, HIP events on `stream` —
 * and writes the fastest to *best (host).  times_ms (host, n_cand floats or
 * NULL) receives each plan's mean launch time.  Every candidate's ids and
 * distances are compared on the device with those of the first candidate of
 * the same gather group (plans of one group sum each distance in the same
 * order, so they must agree bit for bit; across groups FP32 sums may differ
 * in the last place on data whose distances are not exact); any difference
 * returns ANN_EDEVICE.
 * The outputs hold the last candidate's results.  Arguments as ann_search;
 * workspace = ann_autotune_workspace_size(n, dim, nq, k_max) bytes.
 * Synchronises `stream`. */
size_t ann_autotune_workspace_size(int64_t n, int32_t dim, int32_t nq, int32_t k_max);

ann_status ann_autotune_search(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                               int32_t R, const float *queries, int32_t nq,
                               const int32_t *entry_ids, int32_t medoid, const int32_t *k,
                               const int32_t *L, int32_t k_max, int32_t *out_ids,
                               float *out_dist, int32_t *stats, const ann_search_plan *cands,
                               int32_t n_cand, int32_t reps, ann_search_plan *best,
                               float *times_ms, void *workspace, size_t ws_bytes,
                               void *stream);

/* One batch of the query path, described once: the index, the queries and
 * their per-query k and L, the outputs, the plan and the workspaces.  All
 * pointers are device pointers that must stay valid while the batch (or a
 * graph made from it) is used.
 *   entry_ids   nq int32: written by the entry stage, read by the search
 *               stage; NULL (search stage only) = the medoid for every query
 *   model       entry model (host struct, copied) or NULL when no entry stage
 *   entry_ws    ann_entry_workspace_size(model, nq) bytes (entry stage)
 *   search_ws   ann_workspace_size(ANN_OP_SEARCH, n, dim, nq, 0) bytes */
typedef struct ann_query_batch {
    const float *base;
    int64_t n;
    int32_t dim;
    const int32_t *graph;
    int32_t R;
    const float *queries;
    int32_t nq;
    int32_t *entry_ids;
    int32_t medoid;
    const int32_t *k;
    const int32_t *L;
    int32_t k_max;
    int32_t *out_ids;
    float *out_dist;
    int32_t *stats;
    ann_search_plan plan;
    const ann_entry_model *model;
    void *entry_ws;
    size_t entry_ws_bytes;
    void *search_ws;
    size_t search_ws_bytes;
} ann_query_batch;

/* Stages of a batch. */
enum { ANN_STAGE_ENTRY = 1, ANN_STAGE_SEARCH = 2, ANN_STAGE_ALL = 3 };

/* Enqueues the chosen stages of the batch on `stream`: ENTRY =
 * ann_entry_select(model, queries) -> entry_ids; SEARCH = ann_search from
 * entry_ids (or the medoid). */
ann_status ann_query_run(const ann_query_batch *batch, int32_t stages, void *stream);

/* A HIP graph of the chosen stages of a batch (captured once on a private
 * stream; the batch struct and model are copied, the buffers are not).  Each
 * launch replays the same kernels on the buffers' current contents, so new
 * queries written into the same buffers are served by the next launch.
 * The graph holds no memset nodes. */
typedef struct ann_query_graph ann_query_graph;

ann_status ann_query_graph_create(const ann_query_batch *batch, int32_t stages,
                                  ann_query_graph **out);
ann_status ann_query_graph_launch(ann_query_graph *graph, void *stream);
void ann_query_graph_destroy(ann_query_graph *graph);

/* A stream with a hardware queue of its own, for running batches side by
 * side (pipelined batches, serving slots).  Ordinary streams share a small
 * pool of hardware queues, and two streams that land on one queue run their
 * launches one after the other, so whether two batches overlap depends on how
 * many streams the process has created before.  This stream is created with a
 * compute-unit mask naming every compute unit of the current device, which
 * gives it a queue outside that pool; its priority is the default.  *out
 * receives the hipStream_t; release it with ann_stream_destroy (which waits
 * for the stream's pending work).  Errors: ANN_EINVAL for a NULL out,
 * ANN_EDEVICE when the runtime refuses. */
ann_status ann_stream_create(void **out);
void ann_stream_destroy(void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ANN_H */
