// Proximity-graph construction on the GPU: exact kNN candidates, alpha-RNG
// pruning (the triangle-inequality pruning NSG applies; alpha = 1 is MRNG),
// the medoid (navigating node), and connectivity repair so that every node
// is reachable from the medoid and can reach it.
//
//  prune   one wavefront per node; candidates in (d2, id) order; candidate c
//          survives unless a kept o has alpha^2 * d2(o,c) <= d2(p,c), with
//          alpha^2 formed in FP64 from the FP32 alpha and FP64 distances;
//          at most R-2 kept, slots R-2 and R-1 left for repair.
//  medoid  point nearest the mean: FP64 column sums / n, then FP64 squared
//          distance to the mean summed in dimension order without FMA,
//          argmin by (d2, id).
//  repair  forward: BFS from the medoid; the smallest unreached id u is
//          linked from the reached node v with slot R-2 free minimising
//          (d2(u,v), v), and the BFS continues from u.  reverse: BFS over
//          reversed edges; the smallest id w that cannot reach the medoid is
//          linked w -> t, t minimising (d2(w,t), t) over nodes that can.
//          The argmin is read off u's exact kNN list when the list holds an
//          eligible node (the first eligible entry is then the global
//          argmin); otherwise a full scan runs.  The sequential part runs in
//          a single-workgroup driver kernel that returns to the host only
//          for full scans.
#include <hipcub/hipcub.hpp>

#include "common.h"
#include "internal.h"

#include <algorithm>
#include <vector>
#include "knn.h"

namespace ann {



namespace {

// ---------------------------------------------------------------- prune
constexpr int PG = 8;   // lanes per distance

__global__ void __launch_bounds__(256) prune_kernel(const float *base, int64_t n, int dim,
                                                    const int32_t *cand, const double *cand_d2,
                                                    int K, int R, double a2, int32_t *graph)
{
    __shared__ int32_t kept_s[4][64];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + w;
    if (p >= n) return;
    int32_t *kept = kept_s[w];
    const int gi = lane / PG, gl = lane % PG;
    int nk = 0;
    for (int t = 0; t < K && nk < R - 2; ++t) {
        const int32_t c = cand[p * K + t];
        if (c < 0) break;
        const double dpc = cand_d2[p * K + t];
        const float *xc = base + (int64_t)c * dim;
        bool dominated = false;
        for (int b = 0; b < nk && !dominated; b += 64 / PG) {
            const int u = b + gi;
            double acc = 0.0;
            if (u < nk) {
                const float *xo = base + (int64_t)kept[u] * dim;
                for (int j = gl; j < dim; j += PG) {
                    double df = (double)xo[j] - (double)xc[j];
                    acc += df * df;
                }
            }
            for (int o = PG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            bool dom = (u < nk) && (a2 * acc <= dpc);
            dominated = __ballot(dom) != 0;
        }
        if (!dominated) {
            if (lane == 0) kept[nk] = c;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            ++nk;
        }
    }
    for (int s = lane; s < R; s += 64) graph[p * R + s] = s < nk ? kept[s] : -1;
}

// ---------------------------------------------------------------- medoid
constexpr int MED_ROWS = 4096;

__global__ void medoid_colsum_kernel(const float *base, int64_t n, int dim, double *partial)
{
    const int64_t r0 = (int64_t)blockIdx.x * MED_ROWS;
    int64_t r1 = r0 + MED_ROWS;
    if (r1 > n) r1 = n;
    for (int j = threadIdx.x; j < dim; j += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)base[r * dim + j];
        partial[(int64_t)blockIdx.x * dim + j] = s;
    }
}

__global__ void medoid_colmean_kernel(const double *partial, int chunks, int dim, int64_t n, double *mu)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= dim) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * dim + j];
    mu[j] = s / (double)n;
}

struct DKey {
    double v;
    int64_t id;
};

__device__ inline bool dkey_less(const DKey &a, const DKey &b)
{
    return a.v < b.v || (a.v == b.v && a.id < b.id);
}

__device__ double sqdist_to_mean(const float *x, const double *mu, int dim)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        double t = (double)x[j] - mu[j];
        s = s + t * t;
    }
    return s;
}

__device__ inline DKey block_min(DKey k, DKey *sh)
{
    const int t = threadIdx.x;
    sh[t] = k;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s && dkey_less(sh[t + s], sh[t])) sh[t] = sh[t + s];
        __syncthreads();
    }
    DKey r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) medoid_dist_kernel(const float *base, int64_t n, int dim,
                                                          const double *mu, DKey *partial)
{
    __shared__ DKey sh[256];
    DKey best{__longlong_as_double(0x7ff0000000000000ll), 0x7fffffffffffffffll};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        DKey k{sqdist_to_mean(base + i * dim, mu, dim), i};
        if (dkey_less(k, best)) best = k;
    }
    DKey r = block_min(best, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ void argmin_final_kernel(const DKey *partial, int count, DKey *out)
{
    __shared__ DKey sh[256];
    DKey best{__longlong_as_double(0x7ff0000000000000ll), 0x7fffffffffffffffll};
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        if (dkey_less(partial[i], best)) best = partial[i];
    DKey r = block_min(best, sh);
    if (threadIdx.x == 0) *out = r;
}

// ---------------------------------------------------------------- repair
// Full scan: argmin over eligible v of (d2(u, v), v); eligible = mark[v] and
// (slot < 0 or graph[v*R + slot] < 0).
__global__ void __launch_bounds__(256) scan_argmin_kernel(const float *base, int64_t n, int dim,
                                                          const int32_t *graph, int R,
                                                          const int32_t *mark, int slot,
                                                          const int32_t *u_ptr, DKey *partial)
{
    __shared__ DKey sh[256];
    const int64_t u = *u_ptr;
    const float *xu = base + u * dim;
    DKey best{__longlong_as_double(0x7ff0000000000000ll), 0x7fffffffffffffffll};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (!mark[v] || v == u) continue;
        if (slot >= 0 && graph[v * R + slot] >= 0) continue;
        const float *xv = base + v * dim;
        double s = 0.0;
        for (int j = 0; j < dim; ++j) {
            double t = (double)xu[j] - (double)xv[j];
            s += t * t;
        }
        DKey k{s, v};
        if (dkey_less(k, best)) best = k;
    }
    DKey r = block_min(best, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

struct RepairState {
    int64_t head, tail;   // BFS queue window
    int64_t cursor;       // all ids below are marked
    int32_t status;       // 0 running/done, 1 needs full scan for `pending`
    int32_t pending;
    int32_t bridges;
    int32_t phase;        // 0 forward, 1 reverse, 2 done
};

constexpr int DRV = 1024;
constexpr int32_t kNone = 0x7fffffff;

// marks are written by atomics (performed in L2); read them the same way
__device__ inline int32_t ld_mark(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single-workgroup driver.  forward (phase 0) expands over graph rows;
// reverse (phase 1) over the reverse CSR.
__global__ void __launch_bounds__(DRV) repair_driver(int32_t *graph, int64_t n, int R,
                                                     const int32_t *cand, int K, int32_t *mark,
                                                     int32_t *queue, const int64_t *roff,
                                                     const int32_t *radj, RepairState *st,
                                                     int phase)
{
    __shared__ int64_t s_head, s_tail, s_cursor;
    __shared__ int32_t s_found;
    __shared__ int32_t s_u;
    __shared__ int32_t s_pos;
    const int t = threadIdx.x;
    if (t == 0) {
        s_head = st->head;
        s_tail = st->tail;
        s_cursor = st->cursor;
    }
    __syncthreads();
    const int slot = phase == 0 ? R - 2 : R - 1;
    for (;;) {
        // ---- BFS until the queue is empty (level by level)
        while (true) {
            int64_t h = s_head, e = s_tail;
            if (h >= e) break;
            for (int64_t i = h + t; i < e; i += DRV) {
                int32_t v = queue[i];
                if (phase == 0) {
                    for (int s = 0; s < R; ++s) {
                        int32_t w = graph[(int64_t)v * R + s];
                        if (w >= 0 && atomicExch(&mark[w], 1) == 0) {
                            unsigned long long pos = atomicAdd((unsigned long long *)&s_tail, 1ull);
                            queue[pos] = w;
                        }
                    }
                } else {
                    for (int64_t q = roff[v]; q < roff[v + 1]; ++q) {
                        int32_t w = radj[q];
                        if (atomicExch(&mark[w], 1) == 0) {
                            unsigned long long pos = atomicAdd((unsigned long long *)&s_tail, 1ull);
                            queue[pos] = w;
                        }
                    }
                }
            }
            __syncthreads();
            if (t == 0) s_head = e;
            __syncthreads();
        }
        // ---- smallest unmarked id at or after the cursor
        if (t == 0) s_u = kNone;
        __syncthreads();
        while (true) {
            const int64_t c = s_cursor;
            if (c >= n) break;
            const int64_t i = c + t;
            if (i < n && !ld_mark(&mark[i])) atomicMin(&s_u, (int32_t)i);
            __syncthreads();
            if (s_u != kNone) break;
            if (t == 0) s_cursor = c + DRV;
            __syncthreads();
        }
        __syncthreads();
        if (s_u == kNone) {
            if (t == 0) {
                st->status = 0;
                st->head = s_head;
                st->tail = s_tail;
                st->cursor = n;
                st->phase = phase + 1;
            }
            return;
        }
        const int32_t u = s_u;
        // first eligible entry of u's candidate list: each thread tests one
        // position, the smallest eligible position wins (lists end in -1)
        if (t == 0) {
            s_cursor = u;
            s_pos = kNone;
        }
        __syncthreads();
        for (int q = t; q < K; q += DRV) {
            const int32_t v = cand[(int64_t)u * K + q];
            if (v >= 0 && ld_mark(&mark[v]) && (phase == 1 || graph[(int64_t)v * R + slot] < 0))
                atomicMin(&s_pos, q);
        }
        __syncthreads();
        if (t == 0) s_found = s_pos != kNone ? cand[(int64_t)u * K + s_pos] : -1;
        __syncthreads();
        if (s_found < 0) {
            if (t == 0) {
                st->status = 1;
                st->pending = u;
                st->head = s_head;
                st->tail = s_tail;
                st->cursor = u;
                st->phase = phase;
            }
            return;
        }
        if (t == 0) {
            if (phase == 0)
                graph[(int64_t)s_found * R + slot] = u;
            else
                graph[(int64_t)u * R + slot] = s_found;
            atomicExch(&mark[u], 1);
            queue[s_tail] = u;
            s_tail = s_tail + 1;
            st->bridges += 1;
        }
        __syncthreads();
    }
}

// applies the result of a full scan and queues u for the BFS
__global__ void apply_bridge_kernel(int32_t *graph, int R, int32_t *mark, int32_t *queue,
                                    const DKey *best, RepairState *st, int phase)
{
    const int32_t u = st->pending;
    const int32_t v = (int32_t)best->id;
    if (phase == 0)
        graph[(int64_t)v * R + (R - 2)] = u;
    else
        graph[(int64_t)u * R + (R - 1)] = v;
    mark[u] = 1;
    queue[st->tail] = u;
    st->tail += 1;
    st->bridges += 1;
    st->status = 0;
}

__global__ void init_repair_kernel(int32_t *mark, int64_t n, int32_t *queue, int32_t medoid,
                                   RepairState *st, int phase, int reset_bridges)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        mark[i] = (i == medoid) ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        queue[0] = medoid;
        st->head = 0;
        st->tail = 1;
        st->cursor = 0;
        st->status = 0;
        st->pending = -1;
        if (reset_bridges) st->bridges = 0;
        st->phase = phase;
    }
}

__global__ void indeg_kernel(const int32_t *graph, int64_t n, int R, int64_t *cnt)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t w = graph[e];
        if (w >= 0) atomicAdd((unsigned long long *)&cnt[w], 1ull);
    }
}

__global__ void rfill_kernel(const int32_t *graph, int64_t n, int R, const int64_t *off,
                             int64_t *fill, int32_t *adj)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * R;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t w = graph[e];
        if (w >= 0) {
            unsigned long long pos = atomicAdd((unsigned long long *)&fill[w], 1ull);
            adj[off[w] + (int64_t)pos] = (int32_t)(e / R);
        }
    }
}



ann_status run_argmin_scan(const float *base, int64_t n, int dim, const int32_t *graph, int R,
                           const int32_t *mark, int slot, const int32_t *u_ptr, DKey *partial,
                           DKey *best, hipStream_t st)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(scan_argmin_kernel, dim3(blocks), dim3(256), 0, st, base, n, dim, graph, R,
                       mark, slot, u_ptr, partial);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(argmin_final_kernel, dim3(1), dim3(256), 0, st, partial, blocks, best);
    ANN_LAUNCHED();
    return ANN_OK;
}

}  // namespace

size_t scan_temp_bytes(int64_t n)
{
    size_t tmp = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, (int64_t *)nullptr, (int64_t *)nullptr,
                                     (int)(n + 1));
    return tmp;
}


ann_status medoid_run(const float *base, int64_t n, int dim, double *partial_cols, double *mu,
                      void *partial_keys, void *best_key, int32_t *medoid_host, hipStream_t st)
{
    int chunks = (int)((n + MED_ROWS - 1) / MED_ROWS);
    hipLaunchKernelGGL(medoid_colsum_kernel, dim3(chunks), dim3(128), 0, st, base, n, dim, partial_cols);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(medoid_colmean_kernel, dim3((dim + 127) / 128), dim3(128), 0, st, partial_cols,
                       chunks, dim, n, mu);
    ANN_LAUNCHED();
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    DKey *pk = static_cast<DKey *>(partial_keys);
    DKey *bk = static_cast<DKey *>(best_key);
    hipLaunchKernelGGL(medoid_dist_kernel, dim3(blocks), dim3(256), 0, st, base, n, dim, mu, pk);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(argmin_final_kernel, dim3(1), dim3(256), 0, st, pk, blocks, bk);
    ANN_LAUNCHED();
    DKey h{};
    ANN_HIP(hipMemcpyAsync(&h, bk, sizeof(DKey), hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    *medoid_host = (int32_t)h.id;
    return ANN_OK;
}

size_t medoid_ws(int64_t n, int dim)
{
    int chunks = (int)((n + MED_ROWS - 1) / MED_ROWS);
    return round_up((size_t)chunks * dim * 8, 256) + round_up((size_t)dim * 8, 256) +
           round_up(2048 * sizeof(DKey), 256) + round_up(sizeof(DKey), 256);
}

}  // namespace ann

using namespace ann;

namespace ann {
namespace {

// Buffers of the steps after the candidate lists: pruning, medoid, repair.
struct TailBufs {
    int32_t *mark, *queue;
    int64_t *cnt, *off, *fill;
    int32_t *radj;
    void *tmp;
    size_t tmp_bytes;
    double *mu;
    DKey *partial, *best;
    RepairState *rst;
    double *med_cols;    // MED_ROWS-chunk column sums for the medoid
};

size_t tail_ws(int64_t n, int dim, int R)
{
    size_t b = round_up((size_t)n * 4, 256) * 2;                                    // mark, queue
    b += round_up((size_t)(n + 1) * 8, 256) * 3;                                    // cnt, off, fill
    b += round_up((size_t)n * R * 4, 256);                                          // reverse adj
    b += round_up(scan_temp_bytes(n) + 256, 256);
    b += round_up((size_t)dim * 8, 256) + round_up(4096 * sizeof(DKey), 256) * 2;
    b += round_up(sizeof(RepairState), 256);
    b += round_up((size_t)((n + MED_ROWS - 1) / MED_ROWS) * dim * 8, 256);
    return b + 1024;
}

TailBufs take_tail(Carve &cv, int64_t n, int dim, int R)
{
    TailBufs t{};
    t.mark = cv.take<int32_t>((size_t)n);
    t.queue = cv.take<int32_t>((size_t)n);
    t.cnt = cv.take<int64_t>((size_t)n + 1);
    t.off = cv.take<int64_t>((size_t)n + 1);
    t.fill = cv.take<int64_t>((size_t)n + 1);
    t.radj = cv.take<int32_t>((size_t)n * R);
    t.tmp_bytes = scan_temp_bytes(n) + 256;
    t.tmp = cv.take<unsigned char>(t.tmp_bytes);
    t.mu = cv.take<double>((size_t)dim);
    t.partial = cv.take<DKey>(4096);
    t.best = cv.take<DKey>(4096);
    t.rst = cv.take<RepairState>(1);
    t.med_cols = cv.take<double>((size_t)((n + MED_ROWS - 1) / MED_ROWS) * dim);
    return t;
}

// alpha pruning of the candidate lists, medoid, connectivity repair.  Each
// repair bridge is the first eligible entry of the unreached point's
// candidate list, else the argmin over all eligible points (a full scan);
// for lists of global nearest neighbours the two are the same node.
ann_status graph_tail(const float *base, int64_t n, int dim, const int32_t *cand,
                      const double *cd2, int K, int R, float alpha, int32_t *graph,
                      int32_t *medoid, int32_t *bridges, const TailBufs &t, hipStream_t st)
{
    const double a2 = (double)alpha * (double)alpha;
    hipLaunchKernelGGL(prune_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base, n, dim,
                       cand, cd2, K, R, a2, graph);
    ANN_LAUNCHED();
    int32_t med = -1;
    ann_status s = medoid_run(base, n, dim, t.med_cols, t.mu, t.partial, t.best, &med, st);
    if (s != ANN_OK) return s;
    int32_t nb[2] = {0, 0};
    for (int phase = 0; phase < 2; ++phase) {
        if (phase == 1) {
            ANN_HIP(hipMemsetAsync(t.cnt, 0, sizeof(int64_t) * (n + 1), st));
            ANN_HIP(hipMemsetAsync(t.fill, 0, sizeof(int64_t) * (n + 1), st));
            int eb = (int)((n * R + 255) / 256);
            if (eb > 8192) eb = 8192;
            hipLaunchKernelGGL(indeg_kernel, dim3(eb), dim3(256), 0, st, graph, n, R, t.cnt);
            ANN_LAUNCHED();
            size_t tb = t.tmp_bytes;
            ANN_HIP(hipcub::DeviceScan::ExclusiveSum(t.tmp, tb, t.cnt, t.off, (int)(n + 1), st));
            hipLaunchKernelGGL(rfill_kernel, dim3(eb), dim3(256), 0, st, graph, n, R, t.off, t.fill,
                               t.radj);
            ANN_LAUNCHED();
        }
        int ib = (int)((n + 255) / 256);
        if (ib > 4096) ib = 4096;
        hipLaunchKernelGGL(init_repair_kernel, dim3(ib), dim3(256), 0, st, t.mark, n, t.queue, med,
                           t.rst, phase, 1);
        ANN_LAUNCHED();
        for (;;) {
            hipLaunchKernelGGL(repair_driver, dim3(1), dim3(DRV), 0, st, graph, n, R, cand, K,
                               t.mark,
                               t.queue, t.off, t.radj, t.rst, phase);
            ANN_LAUNCHED();
            RepairState h{};
            ANN_HIP(hipMemcpyAsync(&h, t.rst, sizeof(h), hipMemcpyDeviceToHost, st));
            ANN_HIP(hipStreamSynchronize(st));
            if (h.status == 0) {
                nb[phase] = h.bridges;
                break;
            }
            // full scan for rst->pending
            int32_t *u_ptr = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(t.rst) +
                                                         offsetof(RepairState, pending));
            s = run_argmin_scan(base, n, dim, graph, R, t.mark, phase == 0 ? R - 2 : -1, u_ptr,
                                t.partial, t.best, st);
            if (s != ANN_OK) return s;
            hipLaunchKernelGGL(apply_bridge_kernel, dim3(1), dim3(1), 0, st, graph, R, t.mark,
                               t.queue, t.best, t.rst, phase);
            ANN_LAUNCHED();
        }
    }
    *medoid = med;
    if (bridges) {
        bridges[0] = nb[0];
        bridges[1] = nb[1];
    }
    return ANN_OK;
}

// rows[members[r]] -> out row r
__global__ void gather_rows_kernel(const float *base, int dim, const int32_t *members, int64_t m,
                                   float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * dim) return;
    const int64_t r = i / dim;
    out[i] = base[(int64_t)members[r] * dim + (i - r * dim)];
}

// candidate lists of one group's home points (local member indices) -> the
// global lists, -1 / +inf padded
__global__ void scatter_cand_kernel(const int32_t *loc_ids, const double *loc_d2, int Kg,
                                    const int32_t *members, const int32_t *home, int64_t m, int K,
                                    int32_t *cand, double *cd2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * K) return;
    const int64_t r = i / K;
    const int j = (int)(i - r * K);
    const int64_t dst = (int64_t)home[r] * K + j;
    int32_t id = -1;
    double d = __longlong_as_double(0x7ff0000000000000ll);
    if (j < Kg) {
        const int32_t l = loc_ids[r * Kg + j];
        if (l >= 0) {
            id = members[l];
            d = loc_d2[r * Kg + j];
        }
    }
    cand[dst] = id;
    cd2[dst] = d;
}

}  // namespace

size_t build_graph_ws(int64_t n, int dim, int K, int R)
{
    size_t b = knn_workspace(n, n, dim, K);
    b += round_up((size_t)n * K * 4, 256) + round_up((size_t)n * K * 8, 256);  // cand ids, d2
    return b + tail_ws(n, dim, R);
}

size_t group_cand_ws(int dim, int K, int64_t max_mem, int64_t max_home)
{
    size_t b = knn_workspace(max_mem, max_home, dim, K);
    b += round_up((size_t)max_mem * dim * 4, 256) + round_up((size_t)max_home * dim * 4, 256);
    b += round_up((size_t)max_mem * 4, 256) + round_up((size_t)max_home * 4, 256) * 2;
    b += round_up((size_t)max_home * K * 4, 256) + round_up((size_t)max_home * K * 8, 256);
    return b + 1024;
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_build_graph(const float *base, int64_t n, int32_t dim, int32_t knn_k,
                                      int32_t R, float alpha, int32_t *graph, int32_t *medoid,
                                      int32_t *bridges, void *workspace, size_t ws_bytes,
                                      void *stream)
{
    ANN_REQUIRE(base && graph && medoid && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n >= 2 && n <= 0x7FFFFFFF, "n must be in [2, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(R >= 3, "R must be >= 3");
    ANN_SUPPORTED(R <= 64, "R must be <= 64");
    ANN_REQUIRE(knn_k >= R - 2 && knn_k <= 1024, "knn_k must be in [R-2, 1024]");
    ANN_REQUIRE(knn_k <= n - 1, "knn_k must be < n");
    ANN_REQUIRE(alpha >= 1.0f, "alpha must be >= 1");
    ANN_REQUIRE(aligned(base, 16), "base must be 16-byte aligned");
    ANN_REQUIRE(ws_bytes >= ann_workspace_size(ANN_OP_BUILD_GRAPH, n, dim, knn_k, R),
                "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int K = knn_k;
    Carve cv{static_cast<unsigned char *>(workspace)};
    size_t kws = knn_workspace(n, n, dim, K);
    void *knn_ws = cv.take<unsigned char>(kws);
    int32_t *cand = cv.take<int32_t>((size_t)n * K);
    double *cd2 = cv.take<double>((size_t)n * K);
    TailBufs t = take_tail(cv, n, dim, R);
    // exact kNN candidates (self excluded), then pruning, medoid, repair
    ann_status s = knn_run(base, n, dim, base, n, K, true, cand, nullptr, cd2, knn_ws, kws, st, 0);
    if (s != ANN_OK) return s;
    return graph_tail(base, n, dim, cand, cd2, K, R, alpha, graph, medoid, bridges, t, st);
}

namespace {

// Members and home points of every group, each list in id order.
struct GroupLists {
    std::vector<int64_t> ms, hs;          // offsets (n_groups + 1)
    std::vector<int32_t> members, homes;
    int64_t max_mem = 1, max_home = 1;
};

ann_status group_lists(const int32_t *groups_dev, int64_t n, int32_t n_member, int32_t n_groups,
                       hipStream_t st, GroupLists &L)
{
    const size_t nm = (size_t)n_member;
    std::vector<int32_t> lab((size_t)n * nm);
    ANN_HIP(hipMemcpyAsync(lab.data(), groups_dev, sizeof(int32_t) * lab.size(),
                           hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    auto listed_before = [&](int64_t i, size_t c) {
        for (size_t e = 0; e < c; ++e)
            if (lab[(size_t)i * nm + e] == lab[(size_t)i * nm + c]) return true;
        return false;
    };
    L.ms.assign((size_t)n_groups + 1, 0);
    L.hs.assign((size_t)n_groups + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t h = lab[(size_t)i * nm];
        ANN_REQUIRE(h >= 0 && h < n_groups, "home group of point %lld out of range", (long long)i);
        L.hs[(size_t)h + 1]++;
        for (size_t c = 0; c < nm; ++c) {
            const int32_t g = lab[(size_t)i * nm + c];
            ANN_REQUIRE(g >= -1 && g < n_groups, "group label of point %lld out of range",
                        (long long)i);
            if (g >= 0 && !listed_before(i, c)) L.ms[(size_t)g + 1]++;
        }
    }
    for (int g = 0; g < n_groups; ++g) {
        L.max_mem = std::max<int64_t>(L.max_mem, L.ms[(size_t)g + 1]);
        L.max_home = std::max<int64_t>(L.max_home, L.hs[(size_t)g + 1]);
        L.ms[(size_t)g + 1] += L.ms[(size_t)g];
        L.hs[(size_t)g + 1] += L.hs[(size_t)g];
    }
    L.members.resize((size_t)L.ms[(size_t)n_groups]);
    L.homes.resize((size_t)n);
    std::vector<int64_t> mp(L.ms.begin(), L.ms.end() - 1), hp(L.hs.begin(), L.hs.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
        L.homes[(size_t)hp[(size_t)lab[(size_t)i * nm]]++] = (int32_t)i;
        for (size_t c = 0; c < nm; ++c) {
            const int32_t g = lab[(size_t)i * nm + c];
            if (g >= 0 && !listed_before(i, c)) L.members[(size_t)mp[(size_t)g]++] = (int32_t)i;
        }
    }
    return ANN_OK;
}

// candidate lists of the home points of groups [g0, g1)
ann_status group_candidates(const float *base, int dim, int K, const GroupLists &L, int g0, int g1,
                            int32_t *cand, double *cd2, Carve &cv, hipStream_t st)
{
    const size_t kws = knn_workspace(L.max_mem, L.max_home, dim, K);
    void *knn_ws = cv.take<unsigned char>(kws);
    float *mrows = cv.take<float>((size_t)L.max_mem * dim);
    float *hrows = cv.take<float>((size_t)L.max_home * dim);
    int32_t *mem_d = cv.take<int32_t>((size_t)L.max_mem);
    int32_t *home_d = cv.take<int32_t>((size_t)L.max_home);
    int32_t *self_d = cv.take<int32_t>((size_t)L.max_home);
    int32_t *loc_ids = cv.take<int32_t>((size_t)L.max_home * K);
    double *loc_d2 = cv.take<double>((size_t)L.max_home * K);
    std::vector<int32_t> selfc((size_t)L.max_home);
    for (int g = g0; g < g1; ++g) {
        const int64_t m = L.ms[(size_t)g + 1] - L.ms[(size_t)g];
        const int64_t h = L.hs[(size_t)g + 1] - L.hs[(size_t)g];
        if (h == 0) continue;
        const int32_t *mem = L.members.data() + L.ms[(size_t)g];
        const int32_t *hom = L.homes.data() + L.hs[(size_t)g];
        // position of each home point in the member list (both in id order)
        for (int64_t r = 0, e = 0; r < h; ++r) {
            while (mem[e] != hom[r]) ++e;
            selfc[(size_t)r] = (int32_t)e;
        }
        ANN_HIP(hipMemcpyAsync(mem_d, mem, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st));
        ANN_HIP(hipMemcpyAsync(home_d, hom, sizeof(int32_t) * (size_t)h, hipMemcpyHostToDevice, st));
        ANN_HIP(hipMemcpyAsync(self_d, selfc.data(), sizeof(int32_t) * (size_t)h,
                               hipMemcpyHostToDevice, st));
        const int Kg = (int)std::min<int64_t>(K, m - 1);
        if (Kg >= 1) {
            hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((m * dim + 255) / 256)),
                               dim3(256), 0, st, base, dim, mem_d, m, mrows);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((h * dim + 255) / 256)),
                               dim3(256), 0, st, base, dim, home_d, h, hrows);
            ANN_LAUNCHED();
            ann_status s = knn_run(mrows, m, dim, hrows, h, Kg, true, loc_ids, nullptr, loc_d2,
                                   knn_ws, kws, st, 0, self_d);
            if (s != ANN_OK) return s;
        }
        hipLaunchKernelGGL(scatter_cand_kernel, dim3((unsigned)((h * K + 255) / 256)), dim3(256),
                           0, st, loc_ids, loc_d2, Kg, mem_d, home_d, h, K, cand, cd2);
        ANN_LAUNCHED();
        // the staging buffers are rewritten by the next group's copies
        ANN_HIP(hipStreamSynchronize(st));
    }
    return ANN_OK;
}

}  // namespace

#define GROUP_ARGS_OK()                                                                      \
    ANN_REQUIRE(n >= 2 && n <= 0x7FFFFFFF, "n must be in [2, 2^31)");                         \
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");                                                \
    ANN_REQUIRE(knn_k >= 1 && knn_k <= 1024, "knn_k must be in [1, 1024]");                   \
    ANN_REQUIRE(n_member >= 1, "n_member must be >= 1");                                      \
    ANN_REQUIRE(n_groups >= 1, "n_groups must be >= 1");                                      \
    ANN_REQUIRE(aligned(base, 16), "base must be 16-byte aligned")

extern "C" size_t ann_group_candidates_workspace_size(int32_t dim, int32_t knn_k,
                                                      int64_t max_members, int64_t max_home)
{
    if (dim < 1 || knn_k < 1 || max_members < 1 || max_home < 1) return 0;
    return group_cand_ws(dim, knn_k, max_members, max_home);
}

extern "C" ann_status ann_group_candidates(const float *base, int64_t n, int32_t dim, int32_t knn_k,
                                           const int32_t *groups, int32_t n_member,
                                           int32_t n_groups, int32_t g_begin, int32_t g_end,
                                           int32_t *cand, double *cand_d2, void *workspace,
                                           size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && groups && cand && cand_d2 && workspace, "a required pointer is NULL");
    GROUP_ARGS_OK();
    ANN_REQUIRE(g_begin >= 0 && g_begin <= g_end && g_end <= n_groups,
                "group range must satisfy 0 <= g_begin <= g_end <= n_groups");
    hipStream_t st = static_cast<hipStream_t>(stream);
    GroupLists L;
    ann_status s = group_lists(groups, n, n_member, n_groups, st, L);
    if (s != ANN_OK) return s;
    ANN_REQUIRE(ws_bytes >= group_cand_ws(dim, knn_k, L.max_mem, L.max_home),
                "workspace too small (largest member set %lld, largest home set %lld)",
                (long long)L.max_mem, (long long)L.max_home);
    Carve cv{static_cast<unsigned char *>(workspace)};
    return group_candidates(base, dim, knn_k, L, g_begin, g_end, cand, cand_d2, cv, st);
}

extern "C" size_t ann_graph_from_candidates_workspace_size(int64_t n, int32_t dim, int32_t R)
{
    if (n < 2 || dim < 1 || R < 3) return 0;
    return tail_ws(n, dim, R);
}

extern "C" ann_status ann_graph_from_candidates(const float *base, int64_t n, int32_t dim,
                                                const int32_t *cand, const double *cand_d2,
                                                int32_t knn_k, int32_t R, float alpha,
                                                int32_t *graph, int32_t *medoid,
                                                int32_t *bridges, void *workspace,
                                                size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && cand && cand_d2 && graph && medoid && workspace,
                "a required pointer is NULL");
    ANN_REQUIRE(n >= 2 && n <= 0x7FFFFFFF, "n must be in [2, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(R >= 3, "R must be >= 3");
    ANN_SUPPORTED(R <= 64, "R must be <= 64");
    ANN_REQUIRE(knn_k >= R - 2 && knn_k <= 1024, "knn_k must be in [R-2, 1024]");
    ANN_REQUIRE(alpha >= 1.0f, "alpha must be >= 1");
    ANN_REQUIRE(aligned(base, 16), "base must be 16-byte aligned");
    ANN_REQUIRE(ws_bytes >= tail_ws(n, dim, R), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    TailBufs t = take_tail(cv, n, dim, R);
    return graph_tail(base, n, dim, cand, cand_d2, knn_k, R, alpha, graph, medoid, bridges, t, st);
}

extern "C" size_t ann_build_graph_partitioned_workspace_size(int64_t n, int32_t dim,
                                                             int32_t knn_k, int32_t R,
                                                             int64_t max_members, int64_t max_home)
{
    if (n < 2 || dim < 1 || knn_k < 1 || R < 3 || max_members < 1 || max_home < 1) return 0;
    return round_up((size_t)n * knn_k * 4, 256) + round_up((size_t)n * knn_k * 8, 256) +
           std::max(tail_ws(n, dim, R), group_cand_ws(dim, knn_k, max_members, max_home));
}

extern "C" ann_status ann_build_graph_partitioned(const float *base, int64_t n, int32_t dim,
                                                  int32_t knn_k, int32_t R, float alpha,
                                                  const int32_t *groups, int32_t n_member,
                                                  int32_t n_groups, int32_t *graph,
                                                  int32_t *medoid, int32_t *bridges,
                                                  void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && groups && graph && medoid && workspace, "a required pointer is NULL");
    GROUP_ARGS_OK();
    ANN_REQUIRE(R >= 3, "R must be >= 3");
    ANN_SUPPORTED(R <= 64, "R must be <= 64");
    ANN_REQUIRE(knn_k >= R - 2, "knn_k must be >= R-2");
    ANN_REQUIRE(alpha >= 1.0f, "alpha must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    GroupLists L;
    ann_status s = group_lists(groups, n, n_member, n_groups, st, L);
    if (s != ANN_OK) return s;
    ANN_REQUIRE(ws_bytes >= ann_build_graph_partitioned_workspace_size(n, dim, knn_k, R, L.max_mem,
                                                                        L.max_home),
                "workspace too small (largest member set %lld, largest home set %lld)",
                (long long)L.max_mem, (long long)L.max_home);
    const int K = knn_k;
    Carve cv{static_cast<unsigned char *>(workspace)};
    int32_t *cand = cv.take<int32_t>((size_t)n * K);
    double *cd2 = cv.take<double>((size_t)n * K);
    Carve rest = cv;     // the kNN staging and the tail's buffers share what is left
    s = group_candidates(base, dim, K, L, 0, n_groups, cand, cd2, cv, st);
    if (s != ANN_OK) return s;
    TailBufs t = take_tail(rest, n, dim, R);
    return graph_tail(base, n, dim, cand, cd2, K, R, alpha, graph, medoid, bridges, t, st);
}

extern "C" ann_status ann_medoid(const float *base, int64_t n, int32_t dim, int32_t *medoid,
                                 void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && medoid && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(ws_bytes >= medoid_ws(n, dim), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    int chunks = (int)((n + MED_ROWS - 1) / MED_ROWS);
    double *pc = cv.take<double>((size_t)chunks * dim);
    double *mu = cv.take<double>((size_t)dim);
    DKey *partial = cv.take<DKey>(2048);
    DKey *best = cv.take<DKey>(1);
    return medoid_run(base, n, dim, pc, mu, partial, best, medoid, st);
}
