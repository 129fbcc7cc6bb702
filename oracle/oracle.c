/*
 * CPU oracle for the GATE search path (test infrastructure only).
 *
 * This file is a plain, slow, deliberately unoptimised restatement of what the
 * search path computes.  It is compiled with -O2 -ffp-contract=off so that
 * every FP64 expression is evaluated exactly as written (no fused
 * multiply-add).  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load it; the product library never does, and the two share no
 * code.  OpenMP is used only across independent queries / rows, never inside a
 * reduction.
 *
 * Conventions
 *  - squared L2 distance d2(x,y) = sum_j (x_j - y_j)^2 in FP64, j ascending
 *    (the l2 distance of the notation table; squaring is monotone so every
 *    ranking is the one the paper's delta induces);
 *  - every ordering is by the key (value, id): ties go to the smaller id;
 *  - graphs are N x R int32 rows, -1 marks an empty slot.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef int32_t i32;
typedef int64_t i64;

/* ------------------------------------------------------------------------ */
/* Distances (notation table: delta is l2).                                  */

static double d2(const float *x, const float *y, int d)
{
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)x[j] - (double)y[j];
        s = s + t * t;
    }
    return s;
}

static double d2_mixed(const float *x, const double *mu, int d)
{
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)x[j] - mu[j];
        s = s + t * t;
    }
    return s;
}

double oracle_sqdist(const float *x, const float *y, int d) { return d2(x, y, d); }

/* key order: (value, id) */
static int key_less(double a, i32 ia, double b, i32 ib)
{
    return a < b || (a == b && ia < ib);
}

/* ------------------------------------------------------------------------ */
/* Exact k nearest neighbours (recall definition, Eq. 1; graph candidates).  */
/* For query i: all N distances, the k smallest keys (d2, id) in order.       */
/* exclude_self != 0 means query i is base row i and id i is skipped.          */

void oracle_knn(const float *base, i64 n, int d, const float *q, i64 nq, int k,
                int exclude_self, i32 *out_ids, double *out_d2)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (i64 i = 0; i < nq; ++i) {
        i32 *ids = out_ids + i * k;
        double *dd = out_d2 + i * k;
        int cnt = 0;
        for (i64 p = 0; p < n; ++p) {
            if (exclude_self && p == i) continue;
            double v = d2(q + i * d, base + p * d, d);
            if (cnt == k && !key_less(v, (i32)p, dd[k - 1], ids[k - 1])) continue;
            int pos = cnt < k ? cnt : k - 1;
            while (pos > 0 && key_less(v, (i32)p, dd[pos - 1], ids[pos - 1])) {
                dd[pos] = dd[pos - 1];
                ids[pos] = ids[pos - 1];
                --pos;
            }
            dd[pos] = v;
            ids[pos] = (i32)p;
            if (cnt < k) ++cnt;
        }
        for (int t = cnt; t < k; ++t) { ids[t] = -1; dd[t] = INFINITY; }
    }
}

/* ------------------------------------------------------------------------ */
/* Alpha-RNG pruning of a sorted candidate list (the triangle-inequality     */
/* pruning that NSG/MRNG uses; alpha = 1 is the MRNG rule).                   */
/* Candidate c survives iff no already kept o has alpha^2 * d2(o,c) <= d2(p,c) */
/* where alpha^2 is formed in FP64 from the FP32 alpha.  At most R-2 are kept; */
/* slots R-2 and R-1 stay -1 (they are reserved for connectivity repair).      */

void oracle_alpha_prune(const float *base, i64 n, int d, const i32 *cand,
                        const double *cand_d2, int K, int R, float alpha, i32 *graph)
{
    (void)n;
    const double a2 = (double)alpha * (double)alpha;
#pragma omp parallel for schedule(dynamic, 64)
    for (i64 p = 0; p < n; ++p) {
        i32 *row = graph + p * R;
        for (int s = 0; s < R; ++s) row[s] = -1;
        int kept = 0;
        for (int t = 0; t < K && kept < R - 2; ++t) {
            i32 c = cand[p * K + t];
            if (c < 0) break;
            double dpc = cand_d2[p * K + t];
            int dominated = 0;
            for (int u = 0; u < kept && !dominated; ++u) {
                double doc = d2(base + (i64)row[u] * d, base + (i64)c * d, d);
                if (a2 * doc <= dpc) dominated = 1;
            }
            if (!dominated) row[kept++] = c;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Medoid: the base point nearest the dataset mean.  The mean is the FP64     */
/* column sum (taken in row order) divided by n; distances to it are FP64 in  */
/* j order.  argmin over (d2, id).                                            */

static void column_mean(const float *base, i64 n, int d, const i32 *rows, i64 nrows,
                        double *mu)
{
    for (int j = 0; j < d; ++j) mu[j] = 0.0;
    for (i64 r = 0; r < nrows; ++r) {
        const float *x = base + (i64)(rows ? rows[r] : r) * d;
        for (int j = 0; j < d; ++j) mu[j] = mu[j] + (double)x[j];
    }
    for (int j = 0; j < d; ++j) mu[j] = mu[j] / (double)nrows;
    (void)n;
}

i32 oracle_medoid(const float *base, i64 n, int d)
{
    double *mu = (double *)malloc(sizeof(double) * d);
    column_mean(base, n, d, NULL, n, mu);
    double best = INFINITY;
    i32 bi = -1;
    for (i64 i = 0; i < n; ++i) {
        double v = d2_mixed(base + i * d, mu, d);
        if (bi < 0 || key_less(v, (i32)i, best, bi)) { best = v; bi = (i32)i; }
    }
    free(mu);
    return bi;
}

/* ------------------------------------------------------------------------ */
/* Connectivity repair.  The paper relies on NSG's connectivity but does not */
/* say how it is obtained; this is the repair the kNN + alpha graph needs.     */
/*  forward: BFS from the medoid; while a node is unreached take the smallest */
/*           unreached id u, link it from the reached node v with slot R-2    */
/*           still empty that minimises (d2(u,v), v), continue the BFS from u. */
/*  reverse: BFS over reversed edges from the medoid; while a node w cannot   */
/*           reach the medoid (smallest id first), link w -> t where t        */
/*           minimises (d2(w,t), t) over the nodes that can reach it.          */
/* With candidate lists (cand, K per row, -1 ends a row) the bridge of u is   */
/* the first eligible entry of u's list, and the argmin above only when no    */
/* entry is eligible.  For lists that hold u's global nearest neighbours by   */
/* (d2, id) the two rules pick the same node.                                 */
/* Returns the number of forward and reverse bridges through the pointers.    */

static void bfs_from(const i32 *graph, i64 n, int R, i32 src, unsigned char *mark,
                     i32 *queue)
{
    if (mark[src]) return;
    i64 head = 0, tail = 0;
    mark[src] = 1;
    queue[tail++] = src;
    while (head < tail) {
        i32 v = queue[head++];
        for (int s = 0; s < R; ++s) {
            i32 w = graph[(i64)v * R + s];
            if (w >= 0 && !mark[w]) { mark[w] = 1; queue[tail++] = w; }
        }
    }
    (void)n;
}

/* reverse adjacency in CSR form */
static void reverse_csr(const i32 *graph, i64 n, int R, i64 **off_out, i32 **adj_out)
{
    i64 *off = (i64 *)calloc((size_t)n + 1, sizeof(i64));
    for (i64 v = 0; v < n; ++v)
        for (int s = 0; s < R; ++s) {
            i32 w = graph[v * R + s];
            if (w >= 0) off[w + 1]++;
        }
    for (i64 v = 0; v < n; ++v) off[v + 1] += off[v];
    i32 *adj = (i32 *)malloc(sizeof(i32) * (size_t)(off[n] > 0 ? off[n] : 1));
    i64 *fill = (i64 *)malloc(sizeof(i64) * (size_t)n);
    for (i64 v = 0; v < n; ++v) fill[v] = off[v];
    for (i64 v = 0; v < n; ++v)
        for (int s = 0; s < R; ++s) {
            i32 w = graph[v * R + s];
            if (w >= 0) adj[fill[w]++] = (i32)v;
        }
    free(fill);
    *off_out = off;
    *adj_out = adj;
}

static void rbfs_from(const i64 *off, const i32 *adj, i32 src, unsigned char *mark,
                      i32 *queue)
{
    if (mark[src]) return;
    i64 head = 0, tail = 0;
    mark[src] = 1;
    queue[tail++] = src;
    while (head < tail) {
        i32 v = queue[head++];
        for (i64 e = off[v]; e < off[v + 1]; ++e) {
            i32 w = adj[e];
            if (!mark[w]) { mark[w] = 1; queue[tail++] = w; }
        }
    }
}

/* first entry of row u of the candidate lists that passes the test, or -1 */
static i32 first_listed(const i32 *cand, int K, i64 u, const unsigned char *mark,
                        const i32 *graph, int R, int need_free_slot)
{
    if (!cand) return -1;
    for (int q = 0; q < K; ++q) {
        i32 v = cand[u * K + q];
        if (v < 0) break;
        if (mark[v] && (!need_free_slot || graph[(i64)v * R + (R - 2)] < 0)) return v;
    }
    return -1;
}

void oracle_repair(const float *base, i64 n, int d, i32 *graph, int R, i32 medoid,
                   const i32 *cand, int K, i32 *n_forward, i32 *n_reverse)
{
    unsigned char *mark = (unsigned char *)calloc((size_t)n, 1);
    i32 *queue = (i32 *)malloc(sizeof(i32) * (size_t)n);
    int nf = 0, nr = 0;

    bfs_from(graph, n, R, medoid, mark, queue);
    for (i64 u = 0; u < n; ++u) {
        if (mark[u]) continue;
        i32 bv = first_listed(cand, K, u, mark, graph, R, 1);
        if (bv < 0) {
            double best = INFINITY;
            for (i64 v = 0; v < n; ++v) {
                if (!mark[v] || graph[v * R + (R - 2)] >= 0) continue;
                double t = d2(base + u * d, base + v * d, d);
                if (bv < 0 || key_less(t, (i32)v, best, bv)) { best = t; bv = (i32)v; }
            }
        }
        graph[(i64)bv * R + (R - 2)] = (i32)u;
        ++nf;
        bfs_from(graph, n, R, (i32)u, mark, queue);
    }

    i64 *off;
    i32 *adj;
    reverse_csr(graph, n, R, &off, &adj);
    memset(mark, 0, (size_t)n);
    rbfs_from(off, adj, medoid, mark, queue);
    for (i64 w = 0; w < n; ++w) {
        if (mark[w]) continue;
        i32 bt = first_listed(cand, K, w, mark, graph, R, 0);
        if (bt < 0) {
            double best = INFINITY;
            for (i64 t = 0; t < n; ++t) {
                if (!mark[t]) continue;
                double v = d2(base + w * d, base + t * d, d);
                if (bt < 0 || key_less(v, (i32)t, best, bt)) { best = v; bt = (i32)t; }
            }
        }
        graph[w * R + (R - 1)] = bt;
        ++nr;
        /* everything that reaches w now reaches the medoid through w -> bt */
        rbfs_from(off, adj, (i32)w, mark, queue);
    }
    free(off);
    free(adj);
    free(mark);
    free(queue);
    *n_forward = nf;
    *n_reverse = nr;
}

/* ------------------------------------------------------------------------ */
/* Best-first (beam) search, Algorithm 1 read as the standard bounded-pool    */
/* search: a candidate pool of at most L entries kept sorted by (d2, id); the */
/* first k pool entries are the result.  Each loop step expands the best     */
/* not yet expanded pool entry; each of its neighbours not seen before is     */
/* marked visited, its distance computed (one distance computation, "ndc"),  */
/* and it enters the pool if the pool has room or it beats the last entry.    */
/* The search stops when every pool entry has been expanded.                  */
/*                                                                            */
/* Optional outputs:                                                          */
/*   stats[2*i..]  ndc, hops                                                  */
/*   trace[i*trace_cap ..] the ids expanded, in order (-1 padded)             */
/*   visited_out[i*n ..] 0/1 per node (tiny inputs only)                      */

typedef struct { double v; i32 id; int expanded; } entry_t;

static void search_one(const float *base, i64 n, int d, const i32 *graph, int R,
                       const float *q, i32 entry, int k, int L, int k_max,
                       i32 *out_ids, double *out_d2, i64 *stats, i32 *trace,
                       int trace_cap, unsigned char *visited, unsigned char *visited_out)
{
    entry_t *pool = (entry_t *)malloc(sizeof(entry_t) * (size_t)(L + 1));
    i32 *touched = (i32 *)malloc(sizeof(i32) * 1024);
    i64 touched_cap = 1024, ntouched = 0;
    int cnt = 0;
    i64 ndc = 0, hops = 0;

#define VISIT(id_)                                                              \
    do {                                                                        \
        visited[(id_)] = 1;                                                     \
        if (ntouched == touched_cap) {                                          \
            touched_cap *= 2;                                                   \
            touched = (i32 *)realloc(touched, sizeof(i32) * (size_t)touched_cap);\
        }                                                                       \
        touched[ntouched++] = (id_);                                            \
    } while (0)

    /* entry */
    VISIT(entry);
    pool[0].v = d2(q, base + (i64)entry * d, d);
    pool[0].id = entry;
    pool[0].expanded = 0;
    cnt = 1;
    ndc = 1;

    for (;;) {
        int pi = -1;
        for (int t = 0; t < cnt; ++t)
            if (!pool[t].expanded) { pi = t; break; }
        if (pi < 0) break;
        pool[pi].expanded = 1;
        i32 p = pool[pi].id;
        if (trace && hops < trace_cap) trace[hops] = p;
        ++hops;
        for (int s = 0; s < R; ++s) {
            i32 nb = graph[(i64)p * R + s];
            if (nb < 0 || visited[nb]) continue;
            VISIT(nb);
            double v = d2(q, base + (i64)nb * d, d);
            ++ndc;
            if (cnt < L || key_less(v, nb, pool[cnt - 1].v, pool[cnt - 1].id)) {
                int pos = cnt < L ? cnt : L - 1;
                while (pos > 0 && key_less(v, nb, pool[pos - 1].v, pool[pos - 1].id)) {
                    pool[pos] = pool[pos - 1];
                    --pos;
                }
                pool[pos].v = v;
                pool[pos].id = nb;
                pool[pos].expanded = 0;
                if (cnt < L) ++cnt;
            }
        }
    }
#undef VISIT
    for (int t = 0; t < k_max; ++t) {
        if (t < k && t < cnt) { out_ids[t] = pool[t].id; out_d2[t] = pool[t].v; }
        else { out_ids[t] = -1; out_d2[t] = INFINITY; }
    }
    if (stats) { stats[0] = ndc; stats[1] = hops; }
    if (trace)
        for (i64 t = hops; t < trace_cap; ++t) trace[t] = -1;
    if (visited_out)
        for (i64 t = 0; t < ntouched; ++t) visited_out[touched[t]] = 1;
    for (i64 t = 0; t < ntouched; ++t) visited[touched[t]] = 0;
    free(touched);
    free(pool);
    (void)n;
}

void oracle_search(const float *base, i64 n, int d, const i32 *graph, int R,
                   const float *queries, i64 nq, const i32 *entry, const i32 *k,
                   const i32 *L, int k_max, i32 *out_ids, double *out_d2, i64 *stats,
                   i32 *trace, int trace_cap, unsigned char *visited_out, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        unsigned char *visited = (unsigned char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 1)
        for (i64 i = 0; i < nq; ++i) {
            search_one(base, n, d, graph, R, queries + i * d, entry[i], k[i], L[i],
                       k_max, out_ids + i * k_max, out_d2 + i * k_max,
                       stats ? stats + 2 * i : NULL, trace ? trace + i * trace_cap : NULL,
                       trace_cap, visited, visited_out ? visited_out + i * n : NULL);
        }
        free(visited);
    }
}

/* ------------------------------------------------------------------------ */
/* Hub nodes (Definition 3) on Lloyd k-means clusters.                       */
/* init_ids: the n_h starting centroids (given, so both sides start alike).  */
/* Per iteration: assign every point to argmin_c (d2(x, mu_c), c) [FP64, j   */
/* order]; mu_c = FP64 member sum (in id order) / count, an empty cluster    */
/* keeps its centroid; stop once an assignment step changes nothing.        */
/* Hub of cluster c = argmin over members of (d2(x, mu_c), id); an empty     */
/* cluster takes the nearest point that is not yet a hub (cluster order).    */
/* Returns the number of assignment steps run.                               */

/* Definition 3 hubs of given clusters: the member nearest the cluster mean   */
/* by (d2, id); an empty cluster takes the nearest point that is not yet a   */
/* hub (clusters in index order).                                            */
static void hubs_of_clusters(const float *base, i64 n, int d, int nh, const i32 *assign,
                             const double *mu, i32 *hub_ids)
{
    if (n <= 0 || nh <= 0) return;
    double *best = (double *)malloc(sizeof(double) * nh);
    for (int c = 0; c < nh; ++c) { hub_ids[c] = -1; best[c] = INFINITY; }
    for (i64 i = 0; i < n; ++i) {
        int c = assign[i];
        double v = d2_mixed(base + i * d, mu + (i64)c * d, d);
        if (hub_ids[c] < 0 || key_less(v, (i32)i, best[c], hub_ids[c])) { best[c] = v; hub_ids[c] = (i32)i; }
    }
    unsigned char *is_hub = (unsigned char *)calloc((size_t)n, 1);
    for (int c = 0; c < nh; ++c) if (hub_ids[c] >= 0) is_hub[hub_ids[c]] = 1;
    for (int c = 0; c < nh; ++c) {
        if (hub_ids[c] >= 0) continue;
        double bv = INFINITY;
        i32 bi = -1;
        for (i64 i = 0; i < n; ++i) {
            if (is_hub[i]) continue;
            double v = d2_mixed(base + i * d, mu + (i64)c * d, d);
            if (bi < 0 || key_less(v, (i32)i, bv, bi)) { bv = v; bi = (i32)i; }
        }
        hub_ids[c] = bi;
        is_hub[bi] = 1;
    }
    free(is_hub);
    free(best);
}

int oracle_kmeans_hubs(const float *base, i64 n, int d, int nh, int iters,
                       const i32 *init_ids, i32 *hub_ids, double *centroids,
                       i32 *assign, double *objective)
{
    double *mu = centroids;
    for (int c = 0; c < nh; ++c)
        for (int j = 0; j < d; ++j)
            mu[(i64)c * d + j] = (double)base[(i64)init_ids[c] * d + j];
    for (i64 i = 0; i < n; ++i) assign[i] = -1;
    i64 *count = (i64 *)malloc(sizeof(i64) * nh);
    double *sum = (double *)malloc(sizeof(double) * (size_t)nh * d);
    int steps = 0;
    for (int t = 0; t < iters; ++t) {
        int changed = 0;
        double obj = 0.0;
#pragma omp parallel for schedule(static) reduction(| : changed)
        for (i64 i = 0; i < n; ++i) {
            double best = INFINITY;
            int bc = -1;
            for (int c = 0; c < nh; ++c) {
                double v = d2_mixed(base + i * d, mu + (i64)c * d, d);
                if (bc < 0 || key_less(v, c, best, bc)) { best = v; bc = c; }
            }
            if (assign[i] != bc) { changed = 1; assign[i] = bc; }
        }
        ++steps;
        /* objective of this assignment w.r.t. the centroids it used */
        for (i64 i = 0; i < n; ++i) obj += d2_mixed(base + i * d, mu + (i64)assign[i] * d, d);
        if (objective) objective[t] = obj;
        memset(count, 0, sizeof(i64) * nh);
        memset(sum, 0, sizeof(double) * (size_t)nh * d);
        for (i64 i = 0; i < n; ++i) {
            int c = assign[i];
            count[c]++;
            for (int j = 0; j < d; ++j) sum[(i64)c * d + j] = sum[(i64)c * d + j] + (double)base[i * d + j];
        }
        for (int c = 0; c < nh; ++c)
            if (count[c] > 0)
                for (int j = 0; j < d; ++j) mu[(i64)c * d + j] = sum[(i64)c * d + j] / (double)count[c];
        if (!changed) break;
    }
    hubs_of_clusters(base, n, d, nh, assign, mu, hub_ids);
    free(count);
    free(sum);
    return steps;
}

/* ------------------------------------------------------------------------ */
/* Topology features of the hub nodes (feature distillation section).       */
/* The paper samples a subgraph around each hub by a guided walk and embeds   */
/* it with Graph2Vec; here the walk is kept and the embedding is replaced by  */
/* 32 plain statistics of the hub, its neighbourhood and the walk subgraph.   */
/*                                                                            */
/* Guided walk from hub v (max hop h): a FIFO over the subgraph's node list.  */
/* A dequeued node u samples x = max(2, ceil(MinDeg * deg(u) / MaxDeg)) of its */
/* neighbours: the ceil(x/2) nearest and the floor(x/2) farthest by (d2, id)  */
/* (all of them when deg(u) <= x).  Each sampled edge counts; a sampled node  */
/* not yet in the subgraph joins it (while it has fewer than wcap nodes) one  */
/* hop deeper than u and is expanded later if its depth is below h.           */
/* MinDeg / MaxDeg: smallest / largest out-degree over nodes with one.        */
/*                                                                            */
/* Features (nu = mean distance of a node to its first neighbour slot):       */
/*  0 out-degree/R          1 in-degree/mean in-degree                         */
/*  2-6 log2(1 + walk nodes at depth 1..5)   7 log2(1 + walk edges)            */
/*  8-11 mean/min/max/std of dist(v, out-neighbour)/nu                         */
/*  12-15 mean/min/max/std of dist(v, walk node)/nu                            */
/*  16 cluster size/(n/n_h)  17 dist(v, centroid)/nu  18 dist(v, medoid)/nu     */
/*  19 share of walk nodes in another cluster                                  */
/*  20 mean out-degree/R and 21 mean in-degree/mean in-degree of walk nodes     */
/*  22 mean walk-edge length/nu   23 deepest walk depth/h   24-31 zero         */
/* Each column is then standardised across hubs (population std; 0 if none). */

static int cmp_dkey(const void *a, const void *b)
{
    const double *x = (const double *)a, *y = (const double *)b;
    if (x[0] < y[0]) return -1;
    if (x[0] > y[0]) return 1;
    return (x[1] < y[1]) ? -1 : (x[1] > y[1]);
}

static void stats4(const double *v, int m, double *out)
{
    if (m == 0) { out[0] = out[1] = out[2] = out[3] = 0.0; return; }
    double s = 0.0, lo = v[0], hi = v[0];
    for (int i = 0; i < m; ++i) { s += v[i]; if (v[i] < lo) lo = v[i]; if (v[i] > hi) hi = v[i]; }
    double mean = s / m, q = 0.0;
    for (int i = 0; i < m; ++i) q += (v[i] - mean) * (v[i] - mean);
    out[0] = mean; out[1] = lo; out[2] = hi; out[3] = sqrt(q / m);
}

void oracle_hub_features(const float *base, i64 n, int d, const i32 *graph, int R, i32 medoid,
                         const i32 *hub_ids, int nh, const i32 *assign, const double *centroids,
                         int h, int wcap, int standardize, double *feat /* nh x 32 */,
                         i32 *walk_sizes /* nh x 6 */)
{
    int *deg = (int *)calloc((size_t)n, sizeof(int));
    i64 *indeg = (i64 *)calloc((size_t)n, sizeof(i64));
    i64 *csize = (i64 *)calloc((size_t)nh, sizeof(i64));
    int mindeg = 1 << 30, maxdeg = 0;
    double nu = 0.0;
    i64 nu_cnt = 0, edges = 0;
    for (i64 v = 0; v < n; ++v) {
        int c = 0;
        i32 first = -1;
        for (int s = 0; s < R; ++s) {
            i32 w = graph[v * R + s];
            if (w < 0) continue;
            if (first < 0) first = w;
            ++c;
            indeg[w]++;
        }
        deg[v] = c;
        edges += c;
        if (c > 0) {
            if (c < mindeg) mindeg = c;
            if (c > maxdeg) maxdeg = c;
            nu += sqrt(d2(base + v * d, base + (i64)first * d, d));
            nu_cnt++;
        }
        csize[assign[v]]++;
    }
    nu /= (double)nu_cnt;
    const double mean_in = (double)edges / (double)n;

    i32 *S = (i32 *)malloc(sizeof(i32) * (size_t)wcap);
    int *depth = (int *)malloc(sizeof(int) * (size_t)wcap);
    unsigned char *in_s = (unsigned char *)calloc((size_t)n, 1);
    double *buf = (double *)malloc(sizeof(double) * (size_t)(2 * (R > wcap ? R : wcap) + 2));
    double *vals = (double *)malloc(sizeof(double) * (size_t)(wcap > R ? wcap : R));

    for (int c = 0; c < nh; ++c) {
        double *f = feat + (i64)c * 32;
        for (int t = 0; t < 32; ++t) f[t] = 0.0;
        const i32 v = hub_ids[c];
        int ns = 0, head = 0;
        i64 wedges = 0;
        double wlen = 0.0;
        S[ns] = v; depth[ns] = 0; ns++; in_s[v] = 1;
        while (head < ns) {
            int hu = head++;
            if (depth[hu] >= h) continue;
            i32 u = S[hu];
            int du = deg[u];
            int x = (int)(((i64)mindeg * du + maxdeg - 1) / maxdeg);
            if (x < 2) x = 2;
            int m = 0;
            for (int s = 0; s < R; ++s) {
                i32 w = graph[(i64)u * R + s];
                if (w < 0) continue;
                buf[2 * m] = d2(base + (i64)u * d, base + (i64)w * d, d);
                buf[2 * m + 1] = (double)w;
                ++m;
            }
            qsort(buf, (size_t)m, 2 * sizeof(double), cmp_dkey);
            int lo_n = m <= x ? m : (x + 1) / 2;
            int hi_n = m <= x ? 0 : x / 2;
            for (int q = 0; q < lo_n + hi_n; ++q) {
                int idx = q < lo_n ? q : m - hi_n + (q - lo_n);
                i32 w = (i32)buf[2 * idx + 1];
                wedges++;
                wlen += sqrt(buf[2 * idx]);
                if (!in_s[w] && ns < wcap) {
                    in_s[w] = 1;
                    S[ns] = w;
                    depth[ns] = depth[hu] + 1;
                    ns++;
                }
            }
        }
        int cnt_d[6] = {0, 0, 0, 0, 0, 0};
        int maxd = 0;
        for (int q = 0; q < ns; ++q) {
            if (depth[q] <= 5) cnt_d[depth[q]]++;
            if (depth[q] > maxd) maxd = depth[q];
        }
        if (walk_sizes) {
            for (int t = 0; t < 6; ++t) walk_sizes[c * 6 + t] = cnt_d[t];
        }
        f[0] = (double)deg[v] / R;
        f[1] = (double)indeg[v] / mean_in;
        for (int t = 1; t <= 5; ++t) f[1 + t] = log2(1.0 + cnt_d[t]);
        f[7] = log2(1.0 + (double)wedges);
        int m = 0;
        for (int s = 0; s < R; ++s) {
            i32 w = graph[(i64)v * R + s];
            if (w < 0) continue;
            vals[m++] = sqrt(d2(base + (i64)v * d, base + (i64)w * d, d)) / nu;
        }
        stats4(vals, m, f + 8);
        m = 0;
        for (int q = 1; q < ns; ++q) vals[m++] = sqrt(d2(base + (i64)v * d, base + (i64)S[q] * d, d)) / nu;
        stats4(vals, m, f + 12);
        f[16] = (double)csize[c] / ((double)n / nh);
        f[17] = sqrt(d2_mixed(base + (i64)v * d, centroids + (i64)c * d, d)) / nu;
        f[18] = sqrt(d2(base + (i64)v * d, base + (i64)medoid * d, d)) / nu;
        int other = 0;
        double so = 0.0, si = 0.0;
        for (int q = 0; q < ns; ++q) {
            if (q > 0 && assign[S[q]] != c) other++;
            so += deg[S[q]];
            si += (double)indeg[S[q]];
        }
        f[19] = ns > 1 ? (double)other / (ns - 1) : 0.0;
        f[20] = so / ns / R;
        f[21] = si / ns / mean_in;
        f[22] = wedges > 0 ? (wlen / (double)wedges) / nu : 0.0;
        f[23] = (double)maxd / h;
        for (int q = 0; q < ns; ++q) in_s[S[q]] = 0;
    }
    /* standardise columns */
    for (int t = 0; t < 32 && standardize; ++t) {
        double s = 0.0;
        for (int c = 0; c < nh; ++c) s += feat[(i64)c * 32 + t];
        double mean = s / nh, q = 0.0;
        for (int c = 0; c < nh; ++c) {
            double z = feat[(i64)c * 32 + t] - mean;
            q += z * z;
        }
        double sd = sqrt(q / nh);
        for (int c = 0; c < nh; ++c)
            feat[(i64)c * 32 + t] = sd > 0 ? (feat[(i64)c * 32 + t] - mean) / sd : 0.0;
    }
    free(vals); free(buf); free(in_s); free(depth); free(S); free(csize); free(indeg); free(deg);
}

/* ------------------------------------------------------------------------ */
/* Hierarchical balanced k-means hubs (Algorithm 2, Definitions 2 and 3).    */
/* levels = ceil(log_k n_c) with n_c = k^levels exactly.  At each level every */
/* cluster of the previous level (a parent with m members, in id order) is   */
/* split into k children by `iters` iterations of:                           */
/*   - empty children; visit the members in id order, each joining the child */
/*     j minimising d2(x, mu_j) + lambda * (2 (s_j - m/k) + 1), s_j the size  */
/*     child j has reached so far in this pass: the size term of the balance  */
/*     objective of Definition 2 after x joins (the other children's terms    */
/*     are common to every j); ties go to the smaller j;                      */
/*   - mu_j = mean of child j's members (rows in id order); an empty child    */
/*     keeps its centroid.                                                    */
/* Child j starts at the member at position floor((2j + 1) m / (2k)) of the  */
/* parent (a parent without members passes its own centroid on).  Cluster    */
/* p*k + j of a level is child j of cluster p of the level before.  The      */
/* final clusters' hubs follow Definition 3 (hubs_of_clusters).              */

void oracle_hbkm(const float *base, i64 n, int d, int k, int levels, double lambda, int iters,
                 i32 *assign, double *centroids, i32 *hub_ids)
{
    i64 np = 1;                          /* parents at the current level */
    double *pmu = (double *)calloc((size_t)d, sizeof(double));
    i32 *cur = (i32 *)calloc((size_t)n, sizeof(i32));
    i32 *child = (i32 *)malloc(sizeof(i32) * (size_t)n);
    i64 *start = NULL;
    i32 *members = (i32 *)malloc(sizeof(i32) * (size_t)n);
    double *dist = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *mu = NULL;
    for (int l = 1; l <= levels; ++l) {
        const i64 nc = np * k;
        free(start);
        start = (i64 *)calloc((size_t)np + 1, sizeof(i64));
        for (i64 i = 0; i < n; ++i) start[cur[i] + 1]++;
        for (i64 p = 0; p < np; ++p) start[p + 1] += start[p];
        {
            i64 *fill = (i64 *)malloc(sizeof(i64) * (size_t)np);
            for (i64 p = 0; p < np; ++p) fill[p] = start[p];
            for (i64 i = 0; i < n; ++i) members[fill[cur[i]]++] = (i32)i;
            free(fill);
        }
        mu = (double *)malloc(sizeof(double) * (size_t)nc * d);
        i64 *cnt = (i64 *)malloc(sizeof(i64) * (size_t)k);
        for (i64 p = 0; p < np; ++p) {
            const i32 *M = members + start[p];
            const i64 m = start[p + 1] - start[p];
            double *cm = mu + p * k * d;
            for (int j = 0; j < k; ++j)
                for (int c = 0; c < d; ++c)
                    cm[(i64)j * d + c] = m > 0 ? (double)base[(i64)M[(2 * j + 1) * m / (2 * k)] * d + c]
                                               : pmu[p * d + c];
            const double target = (double)m / (double)k;
            for (int t = 0; t < iters; ++t) {
#pragma omp parallel for schedule(static)
                for (i64 r = 0; r < m; ++r)
                    for (int j = 0; j < k; ++j)
                        dist[r * k + j] = d2_mixed(base + (i64)M[r] * d, cm + (i64)j * d, d);
                for (int j = 0; j < k; ++j) cnt[j] = 0;
                for (i64 r = 0; r < m; ++r) {
                    int bj = -1;
                    double bv = INFINITY;
                    for (int j = 0; j < k; ++j) {
                        const double dev = (double)cnt[j] - target;
                        const double pen = lambda * (2.0 * dev + 1.0);
                        const double v = dist[r * k + j] + pen;
                        if (bj < 0 || v < bv) { bv = v; bj = j; }
                    }
                    child[M[r]] = bj;
                    cnt[bj]++;
                }
                for (int j = 0; j < k; ++j) {
                    if (cnt[j] == 0) continue;
                    double *mj = cm + (i64)j * d;
                    for (int c = 0; c < d; ++c) mj[c] = 0.0;
                    for (i64 r = 0; r < m; ++r)
                        if (child[M[r]] == j)
                            for (int c = 0; c < d; ++c) mj[c] = mj[c] + (double)base[(i64)M[r] * d + c];
                    for (int c = 0; c < d; ++c) mj[c] = mj[c] / (double)cnt[j];
                }
            }
            for (i64 r = 0; r < m; ++r) cur[M[r]] = (i32)(p * k + child[M[r]]);
        }
        free(cnt);
        free(pmu);
        pmu = mu;
        np = nc;
    }
    for (i64 i = 0; i < n; ++i) assign[i] = cur[i];
    memcpy(centroids, pmu, sizeof(double) * (size_t)np * d);
    hubs_of_clusters(base, n, d, (int)np, assign, pmu, hub_ids);
    free(pmu);
    free(cur);
    free(child);
    free(start);
    free(members);
    free(dist);
}

/* ------------------------------------------------------------------------ */
/* Hop counts of Definition 4: H(q, V_h) is the length of the shortest path  */
/* along G's (directed) edges from hub h to the nearest neighbour of q.      */
/* One breadth-first search per hub; out[q * nh + h] = H, or 255 when the    */
/* target is unreachable or more than 254 hops away.                         */

void oracle_hop_table(const i32 *graph, i64 n, int R, const i32 *hubs, int nh,
                      const i32 *targets, i64 nq, unsigned char *out)
{
#pragma omp parallel
    {
        int *dist = (int *)malloc(sizeof(int) * (size_t)n);
        i32 *queue = (i32 *)malloc(sizeof(i32) * (size_t)n);
#pragma omp for schedule(dynamic, 1)
        for (int h = 0; h < nh; ++h) {
            for (i64 v = 0; v < n; ++v) dist[v] = -1;
            i64 head = 0, tail = 0;
            dist[hubs[h]] = 0;
            queue[tail++] = hubs[h];
            while (head < tail) {
                i32 v = queue[head++];
                for (int s = 0; s < R; ++s) {
                    i32 w = graph[(i64)v * R + s];
                    if (w >= 0 && dist[w] < 0) { dist[w] = dist[v] + 1; queue[tail++] = w; }
                }
            }
            for (i64 q = 0; q < nq; ++q) {
                int d = dist[targets[q]];
                out[q * nh + h] = (unsigned char)(d < 0 || d > 254 ? 255 : d);
            }
        }
        free(dist);
        free(queue);
    }
}
