// Positive and negative query queues of Definition 4 from a hop table.
//
// With m_h the smallest hop count any query has from hub h, query q is a
// positive of h when H(q, h) <= m_h + t_pos and a negative when it is
// unreachable (255) or H(q, h) >= m_h + t_neg; a hub that reaches no query
// has neither.  Each queue lists its queries in increasing index order; the
// queues are concatenated hub after hub with int64 offsets.
//
// The hop table is nq x n_hubs bytes, row-major (one row per query), so a
// wavefront reading 64 adjacent hubs of one query row is one coalesced
// load.  Work is split into tiles of kChunk queries x 64 hubs: each thread
// owns one hub and kSub consecutive queries of the tile, so the order of the
// queries inside a queue follows from (tile, sub-range, position) and every
// output position is computed, not claimed: the lists come out in the same
// order on every run.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int kHubs = 64;                 // hubs per tile (one wavefront row)
constexpr int kSubs = 4;                  // query sub-ranges per tile (wavefronts)
constexpr int kSub = 64;                  // queries per sub-range
constexpr int kChunk = kSubs * kSub;      // queries per tile
constexpr int kUnreached = 255;

__global__ void queue_min_init_kernel(int32_t *m, int n_hubs)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < n_hubs) m[h] = kUnreached;
}

// m[h] = min over queries of H(q, h) (255 when no query is reachable)
__global__ void __launch_bounds__(256) queue_min_kernel(const uint8_t *H, int64_t nq, int n_hubs,
                                                        int32_t *m)
{
    const int h = blockIdx.y * kHubs + (threadIdx.x & (kHubs - 1));
    if (h >= n_hubs) return;
    const int64_t q0 = (int64_t)blockIdx.x * kChunk + (threadIdx.x / kHubs) * kSub;
    int best = kUnreached;
    for (int i = 0; i < kSub; ++i) {
        const int64_t q = q0 + i;
        if (q >= nq) break;
        const int v = H[q * n_hubs + h];
        best = v < best ? v : best;
    }
    if (best < kUnreached) atomicMin(&m[h], best);
}

struct Rule {
    int t_pos, t_neg;
    __device__ void classify(int v, int mh, bool &pos, bool &neg) const
    {
        const bool any = mh < kUnreached;           // the hub reaches some query
        const bool reach = v < kUnreached;
        pos = any && reach && v <= mh + t_pos;
        neg = any && (!reach || v >= mh + t_neg);
    }
};

// Per tile and hub: the positives and negatives of each sub-range, summed
// over the tile into cnt[tile * n_hubs + h] (pos) and cnt2 (neg).
__global__ void __launch_bounds__(256) queue_count_kernel(const uint8_t *H, int64_t nq, int n_hubs,
                                                          const int32_t *m, Rule rule,
                                                          int32_t *cnt_pos, int32_t *cnt_neg)
{
    __shared__ int sp[kSubs][kHubs], sn[kSubs][kHubs];
    const int lane = threadIdx.x & (kHubs - 1), sub = threadIdx.x / kHubs;
    const int h = blockIdx.y * kHubs + lane;
    int np = 0, nn = 0;
    if (h < n_hubs) {
        const int mh = m[h];
        const int64_t q0 = (int64_t)blockIdx.x * kChunk + sub * kSub;
        for (int i = 0; i < kSub; ++i) {
            const int64_t q = q0 + i;
            if (q >= nq) break;
            bool p, n;
            rule.classify(H[q * n_hubs + h], mh, p, n);
            np += p;
            nn += n;
        }
    }
    sp[sub][lane] = np;
    sn[sub][lane] = nn;
    __syncthreads();
    if (sub == 0 && h < n_hubs) {
        int tp = 0, tn = 0;
        for (int s = 0; s < kSubs; ++s) {
            tp += sp[s][lane];
            tn += sn[s][lane];
        }
        cnt_pos[(int64_t)blockIdx.x * n_hubs + h] = tp;
        cnt_neg[(int64_t)blockIdx.x * n_hubs + h] = tn;
    }
}

// Per hub: exclusive prefix over the tiles (in place) and the hub's totals.
__global__ void queue_tile_scan_kernel(int32_t *cnt_pos, int32_t *cnt_neg, int tiles, int n_hubs,
                                       int64_t *tot_pos, int64_t *tot_neg)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_hubs) return;
    int64_t ap = 0, an = 0;
    for (int t = 0; t < tiles; ++t) {
        const int64_t i = (int64_t)t * n_hubs + h;
        const int32_t p = cnt_pos[i], n = cnt_neg[i];
        cnt_pos[i] = (int32_t)ap;     // a hub's queue within one tile range stays < nq < 2^31
        cnt_neg[i] = (int32_t)an;
        ap += p;
        an += n;
    }
    tot_pos[h] = ap;
    tot_neg[h] = an;
}

// off[0] = 0, off[h + 1] = off[h] + tot[h] for both queues (one workgroup;
// each thread sums a contiguous block of hubs, then a scan over the threads).
__global__ void __launch_bounds__(1024) queue_offsets_kernel(const int64_t *tot_pos,
                                                             const int64_t *tot_neg, int n_hubs,
                                                             int64_t *pos_off, int64_t *neg_off)
{
    __shared__ int64_t bp[1024], bn[1024];
    const int t = threadIdx.x;
    const int per = (n_hubs + 1023) / 1024;
    const int lo = t * per, hi = min(n_hubs, lo + per);
    int64_t sp = 0, sn = 0;
    for (int h = lo; h < hi; ++h) {
        sp += tot_pos[h];
        sn += tot_neg[h];
    }
    bp[t] = sp;
    bn[t] = sn;
    __syncthreads();
    if (t == 0) {
        int64_t ap = 0, an = 0;
        for (int i = 0; i < 1024; ++i) {
            const int64_t p = bp[i], n = bn[i];
            bp[i] = ap;
            bn[i] = an;
            ap += p;
            an += n;
        }
        pos_off[n_hubs] = ap;
        neg_off[n_hubs] = an;
    }
    __syncthreads();
    int64_t ap = bp[t], an = bn[t];
    for (int h = lo; h < hi; ++h) {
        pos_off[h] = ap;
        neg_off[h] = an;
        ap += tot_pos[h];
        an += tot_neg[h];
    }
}

// Writes each hub's queries of the tile at off[h] + tile prefix + the
// counts of the earlier sub-ranges + the rank inside the sub-range.
__global__ void __launch_bounds__(256) queue_fill_kernel(const uint8_t *H, int64_t nq, int n_hubs,
                                                         const int32_t *m, Rule rule,
                                                         const int32_t *pre_pos,
                                                         const int32_t *pre_neg,
                                                         const int64_t *pos_off,
                                                         const int64_t *neg_off, int32_t *pos_q,
                                                         int32_t *neg_q)
{
    __shared__ int sp[kSubs][kHubs], sn[kSubs][kHubs];
    const int lane = threadIdx.x & (kHubs - 1), sub = threadIdx.x / kHubs;
    const int h = blockIdx.y * kHubs + lane;
    const int64_t q0 = (int64_t)blockIdx.x * kChunk + sub * kSub;
    const int mh = h < n_hubs ? m[h] : kUnreached;
    int np = 0, nn = 0;
    if (h < n_hubs) {
        for (int i = 0; i < kSub; ++i) {
            const int64_t q = q0 + i;
            if (q >= nq) break;
            bool p, n;
            rule.classify(H[q * n_hubs + h], mh, p, n);
            np += p;
            nn += n;
        }
    }
    sp[sub][lane] = np;
    sn[sub][lane] = nn;
    __syncthreads();
    if (h >= n_hubs) return;
    int64_t wp = pos_off[h] + pre_pos[(int64_t)blockIdx.x * n_hubs + h];
    int64_t wn = neg_off[h] + pre_neg[(int64_t)blockIdx.x * n_hubs + h];
    for (int s = 0; s < sub; ++s) {
        wp += sp[s][lane];
        wn += sn[s][lane];
    }
    for (int i = 0; i < kSub; ++i) {
        const int64_t q = q0 + i;
        if (q >= nq) break;
        bool p, n;
        rule.classify(H[q * n_hubs + h], mh, p, n);
        if (p) pos_q[wp++] = (int32_t)q;
        if (n) neg_q[wn++] = (int32_t)q;
    }
}

struct QueueWs {
    int32_t *m, *cnt_pos, *cnt_neg;
    int64_t *tot_pos, *tot_neg;
};

size_t queue_ws_bytes(int64_t nq, int n_hubs)
{
    const int64_t tiles = (nq + kChunk - 1) / kChunk;
    return round_up((size_t)n_hubs * 4, 256) + 2 * round_up((size_t)(tiles * n_hubs) * 4, 256) +
           2 * round_up((size_t)n_hubs * 8, 256);
}

QueueWs queue_ws(int64_t nq, int n_hubs, void *base)
{
    const int64_t tiles = (nq + kChunk - 1) / kChunk;
    Carve cv{static_cast<unsigned char *>(base)};
    QueueWs x{};
    x.m = cv.take<int32_t>((size_t)n_hubs);
    x.cnt_pos = cv.take<int32_t>((size_t)(tiles * n_hubs));
    x.cnt_neg = cv.take<int32_t>((size_t)(tiles * n_hubs));
    x.tot_pos = cv.take<int64_t>((size_t)n_hubs);
    x.tot_neg = cv.take<int64_t>((size_t)n_hubs);
    return x;
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" size_t ann_make_queues_workspace_size(int64_t nq, int32_t n_hubs)
{
    if (nq < 1 || n_hubs < 1) return 256;
    return queue_ws_bytes(nq, n_hubs);
}

extern "C" ann_status ann_make_queues(const uint8_t *hops, int64_t nq, int32_t n_hubs, int32_t t_pos,
                                      int32_t t_neg, int64_t *pos_off, int64_t *neg_off,
                                      int32_t *pos_q, int64_t pos_cap, int32_t *neg_q,
                                      int64_t neg_cap, int64_t *totals, void *workspace,
                                      size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(hops && pos_off && neg_off && totals && workspace, "a required pointer is NULL");
    ANN_REQUIRE(nq >= 1 && nq <= 0x7FFFFFFF, "nq must be in [1, 2^31)");
    ANN_REQUIRE(n_hubs >= 1 && n_hubs <= (1 << 20), "n_hubs must be in [1, 2^20]");
    ANN_REQUIRE(t_pos >= 0 && t_neg >= 0, "t_pos and t_neg must be >= 0");
    ANN_REQUIRE(pos_cap >= 0 && neg_cap >= 0, "capacities must be >= 0");
    ANN_REQUIRE((pos_cap == 0 || pos_q) && (neg_cap == 0 || neg_q),
                "a queue buffer is NULL but its capacity is not 0");
    ANN_REQUIRE(ws_bytes >= ann_make_queues_workspace_size(nq, n_hubs), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const QueueWs w = queue_ws(nq, n_hubs, workspace);
    const int tiles = (int)((nq + kChunk - 1) / kChunk);
    const dim3 grid((unsigned)tiles, (unsigned)((n_hubs + kHubs - 1) / kHubs));
    const Rule rule{t_pos, t_neg};
    hipLaunchKernelGGL(queue_min_init_kernel, dim3((n_hubs + 255) / 256), dim3(256), 0, st, w.m,
                       n_hubs);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(queue_min_kernel, grid, dim3(256), 0, st, hops, nq, n_hubs, w.m);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(queue_count_kernel, grid, dim3(256), 0, st, hops, nq, n_hubs, w.m, rule,
                       w.cnt_pos, w.cnt_neg);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(queue_tile_scan_kernel, dim3((n_hubs + 255) / 256), dim3(256), 0, st,
                       w.cnt_pos, w.cnt_neg, tiles, n_hubs, w.tot_pos, w.tot_neg);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(queue_offsets_kernel, dim3(1), dim3(1024), 0, st, w.tot_pos, w.tot_neg,
                       n_hubs, pos_off, neg_off);
    ANN_LAUNCHED();
    ANN_HIP(hipMemcpyAsync(&totals[0], pos_off + n_hubs, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ANN_HIP(hipMemcpyAsync(&totals[1], neg_off + n_hubs, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    if (totals[0] > pos_cap || totals[1] > neg_cap)
        return fail(ANN_ENOMEM, "queues need %lld positive and %lld negative slots (capacity %lld, %lld)",
                    (long long)totals[0], (long long)totals[1], (long long)pos_cap,
                    (long long)neg_cap);
    hipLaunchKernelGGL(queue_fill_kernel, grid, dim3(256), 0, st, hops, nq, n_hubs, w.m, rule,
                       w.cnt_pos, w.cnt_neg, pos_off, neg_off, pos_q, neg_q);
    ANN_LAUNCHED();
    return ANN_OK;
}
