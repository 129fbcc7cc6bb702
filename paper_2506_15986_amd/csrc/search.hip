// Batched best-first beam search on a proximity graph (Algorithm 1 read as
// the bounded-pool search), one wavefront per query, persistent grid.
//
// Per hop a wavefront: picks the best unexpanded pool entry (ballot over the
// sorted pool), loads its adjacency row with one coalesced load, test-and-sets
// every neighbour in the LDS visited filter, compacts the unseen ones (slot
// order is kept), gathers their vectors in groups of G lanes with 16-byte
// loads (G*16 contiguous bytes per group and instruction), reduces the FP32
// (or FP64) squared L2 distance with lane shuffles, and merges the new keys
// into the pool.  For FP32 keys and pools of up to 256 entries every lane
// holds its pool entries as 64-bit words and one pass over the new keys
// counts, per compare mask, each new key's insertion point and rank and each
// entry's shift, and the merged pool is written back in place; otherwise
// insertion points come from binary searches, the old entries' places from
// occupancy bits, and the merge goes to a second (ping-pong) buffer.  Keys are
// (distance, id), so ties go to the smaller id.
//
// When the visited filter is a hash table that had to drop an id, a dropped
// node may be seen again.  Its key is recomputed bit-identically, so it is
// either still in the pool (equal to the entry at its insertion point, and
// dropped as a duplicate) or it was rejected or evicted while the pool was full, and
// since the pool's last key only decreases once the pool is full it is
// rejected again: the expansion order and results are those of an exact
// visited set; only the executed distance count grows.
#include "beam.h"
#include "common.h"
#include "internal.h"
#include "search_core.h"

namespace ann {
namespace {

using namespace beam;

template <int G, int CPL, bool F64, int FILT>
__global__ void __launch_bounds__(256) search_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    using S = Searcher<G, CPL, F64, FILT>;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    S s;
    s.setup(smem + (size_t)wave * a.wave_lds, a.pool_cap, a.visited_log2, a.filter, a.n, a.base,
            a.dim, a.graph, a.R);
    for (;;) {
        int slot = 0;
        if (lane == 0) slot = (int)atomicAdd(a.counter, 1u);
        slot = __shfl(slot, 0);
        if (slot >= a.nq) break;
        const int qi = a.order ? a.order[slot] : slot;
        if (qi < 0 || qi >= a.nq) continue;
        const int kq = a.k[qi];
        const int Lq = a.L[qi];
        const int entry = a.entry ? a.entry[qi] : a.medoid;
        int32_t *oid = a.out_ids + (size_t)qi * a.k_max;
        float *odist = a.out_dist + (size_t)qi * a.k_max;
        int32_t *trace = a.trace ? a.trace + (size_t)qi * a.trace_cap : nullptr;
        if (kq < 1 || kq > Lq || Lq > a.pool_cap || kq > a.k_max || entry < 0 ||
            (int64_t)entry >= a.n) {
            for (int t = lane; t < a.k_max; t += 64) {
                oid[t] = -1;
                odist[t] = __int_as_float(0x7f800000);
            }
            for (int t = lane; trace && t < a.trace_cap; t += 64) trace[t] = -1;
            if (a.stats && lane == 0) {
                int32_t *st = a.stats + (size_t)qi * 4;
                st[0] = 0; st[1] = 0; st[2] = 0; st[3] = 2;
            }
            continue;
        }
        s.load_query(a.queries + (size_t)qi * a.dim);
        SearchResult r = s.run((uint32_t)entry, Lq, trace, a.trace_cap);
        s.write_topk(kq, a.k_max, oid, odist);
        for (int t = (int)r.hops + lane; trace && t < a.trace_cap; t += 64) trace[t] = -1;
        if (a.stats && lane == 0) {
            int32_t *st = a.stats + (size_t)qi * 4;
            st[0] = r.ndc_exec - r.dups;
            st[1] = r.ndc_exec;
            st[2] = r.hops;
            st[3] = r.lost ? 1 : 0;
        }
    }
}

// ---- widest-expected-first order.  A query whose entry lies far from it,
// or whose beam is wide, usually needs more hops; a persistent launch that
// starts such queries last waits for them at the end.  The queries are
// therefore taken in order of L times the FP32 squared distance from the
// query to its entry vector, largest first, binned by the top 13 bits of
// that value (exponent and 4 mantissa bits: bins 4.4 % wide) with a counting
// sort in one workgroup.  Results do not depend on the order; only the
// launch's tail does.  (Within a bin the order follows LDS atomics and may
// vary between runs.)
constexpr int ORDER_BITS = 13;
constexpr int ORDER_BINS = 1 << ORDER_BITS;
constexpr int ORDER_PER_THREAD = ORDER_BINS / 1024;

// one wavefront per query: its bin of L x distance to the entry vector
__global__ void __launch_bounds__(256) order_key_kernel(const float *base, int64_t n, int dim,
                                                        const float *queries, int nq,
                                                        const int32_t *entry, int medoid,
                                                        const int32_t *L, uint32_t *key)
{
    const int q = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= nq) return;
    const int e = entry ? entry[q] : medoid;
    float acc = 0.0f;
    if (e >= 0 && (int64_t)e < n) {
        const float *x = base + (size_t)e * dim;
        const float *y = queries + (size_t)q * dim;
        for (int j = lane; j < dim; j += 64) {
            const float d = y[j] - x[j];
            acc += d * d;
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const int Lq = L[q];
        key[q] = __float_as_uint(acc * (float)(Lq > 0 ? Lq : 0)) >> (32 - ORDER_BITS);
    }
}

// counting sort of the bins, largest first, in one workgroup: counts in LDS,
// a descending exclusive scan (thread t owns places ORDER_PER_THREAD * t ...
// of the descending bin list), then each query takes the next place of its bin.
// It also zeroes the search's work counter (it runs just before the search on
// the same stream, so the search launch needs no reset of its own).
__global__ void __launch_bounds__(1024) order_sort_kernel(const uint32_t *key, int nq,
                                                          int32_t *order, uint32_t *counter)
{
    __shared__ uint32_t hist[ORDER_BINS];
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    if (t == 0) *counter = 0u;
    for (int i = t; i < ORDER_BINS; i += 1024) hist[i] = 0u;
    __syncthreads();
    for (int q = t; q < nq; q += 1024) atomicAdd(&hist[key[q]], 1u);
    __syncthreads();
    uint32_t c[ORDER_PER_THREAD], sum = 0u;
    for (int i = 0; i < ORDER_PER_THREAD; ++i) {
        c[i] = hist[ORDER_BINS - 1 - (ORDER_PER_THREAD * t + i)];
        sum += c[i];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0u;
    for (int i = 0; i < ORDER_PER_THREAD; ++i) {
        hist[ORDER_BINS - 1 - (ORDER_PER_THREAD * t + i)] = run;
        run += c[i];
    }
    __syncthreads();
    for (int q = t; q < nq; q += 1024) order[atomicAdd(&hist[key[q]], 1u)] = q;
}

template <int G, int CPL, bool F64, int FILT>
ann_status launch_one(const SearchArgs &a, int blocks, int wpb, hipStream_t st)
{
    auto kern = search_kernel<G, CPL, F64, FILT>;
    size_t lds = (size_t)wpb * a.wave_lds;
    if (lds > 65536) ANN_HIP(hipFuncSetAttribute((const void *)kern,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds));
    if (blocks <= 0) {
        int per_cu = 0;
        ANN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds));
        if (per_cu < 1) return fail(ANN_ENOTSUP, "search plan does not fit on a CU (%zu B LDS)", lds);
        blocks = per_cu * device_cus();
    }
    int need = (a.nq + wpb - 1) / wpb;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    if (!a.order) {   // with the query-order pre-pass its sort kernel zeroed it
        ann_status rs = reset_work_counter(a.counter, st);
        if (rs != ANN_OK) return rs;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a);
    ANN_LAUNCHED();
    return ANN_OK;
}

template <int G, int CPL, bool F64>
ann_status launch_search(const SearchArgs &a, int blocks, int wpb, hipStream_t st)
{
    switch (a.filter.kind) {
    case kBitset: return launch_one<G, CPL, F64, kBitset>(a, blocks, wpb, st);
    case kTag16: return launch_one<G, CPL, F64, kTag16>(a, blocks, wpb, st);
    case kTag12: return launch_one<G, CPL, F64, kTag12>(a, blocks, wpb, st);
    case kId32: return launch_one<G, CPL, F64, kId32>(a, blocks, wpb, st);
    default: break;
    }
    return fail(ANN_ENOTSUP, "unknown filter form %d", a.filter.kind);
}

template <bool F64>
ann_status dispatch(const SearchArgs &a, int group, int blocks, int wpb, hipStream_t st)
{
    const int chunks = a.dim / 4;
    if (group == 4) {
        int cpl = (chunks + 3) / 4;
        if (cpl <= 1) return launch_search<4, 1, F64>(a, blocks, wpb, st);
        if (cpl <= 2) return launch_search<4, 2, F64>(a, blocks, wpb, st);
        if (cpl <= 4) return launch_search<4, 4, F64>(a, blocks, wpb, st);
        return fail(ANN_ENOTSUP, "group 4 supports dim <= 64 (got %d)", a.dim);
    }
    if (group == 8) {
        int cpl = (chunks + 7) / 8;
        switch (cpl) {
        case 1: return launch_search<8, 1, F64>(a, blocks, wpb, st);
        case 2: return launch_search<8, 2, F64>(a, blocks, wpb, st);
        case 3: return launch_search<8, 3, F64>(a, blocks, wpb, st);
        case 4: return launch_search<8, 4, F64>(a, blocks, wpb, st);
        default: break;
        }
        return fail(ANN_ENOTSUP, "group 8 supports dim <= 128 (got %d)", a.dim);
    }
    int cpl = (chunks + 15) / 16;
    if (cpl <= 1) return launch_search<16, 1, F64>(a, blocks, wpb, st);
    if (cpl <= 2) return launch_search<16, 2, F64>(a, blocks, wpb, st);
    if (cpl <= 4) return launch_search<16, 4, F64>(a, blocks, wpb, st);
    if (cpl <= 8) return launch_search<16, 8, F64>(a, blocks, wpb, st);
    if (cpl <= 15) return launch_search<16, 15, F64>(a, blocks, wpb, st);
    if (cpl <= 16) return launch_search<16, 16, F64>(a, blocks, wpb, st);
    return fail(ANN_ENOTSUP, "dim %d exceeds 1024", a.dim);
}

}  // namespace

ann_status validate_plan(const ann_search_plan &p)
{
    ANN_REQUIRE(p.pool_cap >= 1 && p.pool_cap <= 1024, "plan.pool_cap must be in [1,1024]");
    ANN_REQUIRE(p.visited_log2 >= 8 && p.visited_log2 <= 14, "plan.visited_log2 must be in [8,14]");
    ANN_REQUIRE(p.group == 4 || p.group == 8 || p.group == 16, "plan.group must be 4, 8 or 16");
    ANN_REQUIRE(p.waves_per_block == 1 || p.waves_per_block == 2 || p.waves_per_block == 4,
                "plan.waves_per_block must be 1, 2 or 4");
    ANN_REQUIRE(p.blocks >= 0, "plan.blocks must be >= 0");
    ANN_REQUIRE(p.fp64 == 0 || p.fp64 == 1, "plan.fp64 must be 0 or 1");
    ANN_REQUIRE(p.filter >= ANN_FILTER_AUTO && p.filter <= ANN_FILTER_TAG12,
                "plan.filter must be one of ANN_FILTER_*");
    ANN_REQUIRE(p.waves_per_query >= 0 && p.waves_per_query <= 4 && p.waves_per_query != 3,
                "plan.waves_per_query must be 1, 2 or 4 (0 = 1)");
    ANN_REQUIRE(p.waves_per_query <= 1 || p.waves_per_block == p.waves_per_query,
                "plan.waves_per_block must equal waves_per_query when it is above 1");
    ANN_SUPPORTED(p.waves_per_query <= 1 || (p.group == 16 && p.fp64 == 0),
                  "several waves per query need group 16 and FP32");
    ANN_REQUIRE(p.query_order == ANN_ORDER_WIDEST_FIRST || p.query_order == ANN_ORDER_AS_GIVEN,
                "plan.query_order must be one of ANN_ORDER_*");
    return ANN_OK;
}

ann_status search_filter(const ann_search_plan &p, int64_t n, FilterShape &f)
{
    if (!filter_shape(p.filter, p.visited_log2, n, f))
        return fail(ANN_ENOTSUP, "plan.filter %d cannot hold %lld ids with visited_log2 %d",
                    p.filter, (long long)n, p.visited_log2);
    return ANN_OK;
}

size_t search_wave_lds(const ann_search_plan &p, int64_t n, int dim)
{
    FilterShape f{};
    if (!filter_shape(p.filter, p.visited_log2, n, f)) return 0;
    return wave_lds_bytes(p.pool_cap, f, p.fp64 != 0, dim);
}

size_t search_ws_bytes(int64_t nq)
{
    if (nq <= 1) return 256;
    return 256 + 2 * round_up((size_t)nq * 4, 256);
}

ann_status search_launch(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                         int32_t R, const float *queries, int32_t nq, const int32_t *entry_ids,
                         int32_t medoid, const int32_t *k, const int32_t *L, int32_t k_max,
                         int32_t *out_ids, float *out_dist, int32_t *stats, int32_t *trace,
                         int32_t trace_cap, const ann_search_plan &p, uint32_t *counter,
                         hipStream_t st, bool widest_first)
{
    SearchArgs a{};
    a.base = base;
    a.n = n;
    a.dim = dim;
    a.graph = graph;
    a.R = R;
    a.queries = queries;
    a.nq = nq;
    a.entry = entry_ids;
    a.medoid = medoid;
    a.k = k;
    a.L = L;
    a.k_max = k_max;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.stats = stats;
    a.trace = trace;
    a.trace_cap = trace ? trace_cap : 0;
    a.pool_cap = p.pool_cap;
    a.visited_log2 = p.visited_log2;
    a.counter = counter;
    {
        ann_status fs = search_filter(p, n, a.filter);
        if (fs != ANN_OK) return fs;
    }
    a.wave_lds = wave_lds_bytes(p.pool_cap, a.filter, p.fp64 != 0, dim);
    a.order = nullptr;
    if (widest_first && p.query_order == ANN_ORDER_WIDEST_FIRST && nq > 1) {
        // the workspace after the counter: order, keys
        Carve cv{reinterpret_cast<unsigned char *>(counter) + 256};
        int32_t *order = cv.take<int32_t>((size_t)nq);
        uint32_t *key = cv.take<uint32_t>((size_t)nq);
        hipLaunchKernelGGL(order_key_kernel, dim3((nq + 3) / 4), dim3(256), 0, st, base, n, dim,
                           queries, nq, entry_ids, medoid, L, key);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(order_sort_kernel, dim3(1), dim3(1024), 0, st, key, nq, order, counter);
        ANN_LAUNCHED();
        a.order = order;
    }
    if (p.waves_per_query > 1) return launch_search_mw(a, p.waves_per_query, p.blocks, st);
    if (p.fp64) return dispatch<true>(a, p.group, p.blocks, p.waves_per_block, st);
    return dispatch<false>(a, p.group, p.blocks, p.waves_per_block, st);
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_default_plan(int64_t n, int32_t dim, int32_t R, int32_t L_max,
                                       ann_search_plan *plan)
{
    ANN_REQUIRE(plan != nullptr, "plan is NULL");
    ANN_REQUIRE(n >= 1 && dim >= 1 && R >= 1 && L_max >= 1, "n, dim, R, L_max must be >= 1");
    ANN_SUPPORTED(L_max <= 1024, "L_max %d exceeds 1024", L_max);
    ann_search_plan p{};
    p.pool_cap = (L_max + 15) / 16 * 16;
    p.visited_log2 = 12;
    p.filter = ANN_FILTER_AUTO;
    p.waves_per_query = 1;
    p.group = dim <= 128 ? 8 : 16;
    p.waves_per_block = 1;
    p.blocks = 0;
    p.fp64 = 0;
    p.query_order = ANN_ORDER_WIDEST_FIRST;
    (void)R;
    *plan = p;
    return ANN_OK;
}

namespace ann {

ann_status search_check(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                        int32_t R, const float *queries, int32_t nq, const int32_t *entry_ids,
                        int32_t medoid, const int32_t *k, const int32_t *L, int32_t k_max,
                        int32_t *out_ids, float *out_dist, int32_t *trace, int32_t trace_cap,
                        const ann_search_plan *plan, void *workspace, size_t ws_bytes,
                        ann_search_plan &p)
{
    ANN_REQUIRE(base && graph && workspace, "a required pointer is NULL");
    ANN_REQUIRE(nq == 0 || (queries && k && L && out_ids && out_dist),
                "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_SUPPORTED(dim % 4 == 0, "dim must be a multiple of 4 (got %d)", dim);
    ANN_SUPPORTED(dim <= 1024, "dim must be <= 1024 (got %d)", dim);
    ANN_REQUIRE(R >= 1, "R must be >= 1");
    ANN_SUPPORTED(R <= 64, "R must be <= 64 (got %d)", R);
    ANN_REQUIRE(nq >= 0, "nq must be >= 0");
    ANN_REQUIRE(k_max >= 1, "k_max must be >= 1");
    ANN_REQUIRE(entry_ids != nullptr || (medoid >= 0 && (int64_t)medoid < n),
                "medoid out of range");
    ANN_REQUIRE(aligned(base, 16) && aligned(queries, 16), "base/queries must be 16-byte aligned");
    ANN_REQUIRE(trace == nullptr || trace_cap >= 1, "trace_cap must be >= 1 with a trace buffer");
    ANN_REQUIRE(ws_bytes >= ann_workspace_size(ANN_OP_SEARCH, n, dim, nq, 0),
                "workspace too small");
    if (plan) {
        p = *plan;
    } else {
        ann_status s = ann_default_plan(n, dim, R, 256, &p);
        if (s != ANN_OK) return s;
    }
    ann_status s = validate_plan(p);
    if (s != ANN_OK) return s;
    ANN_SUPPORTED(p.group != 4 || dim <= 64, "group 4 supports dim <= 64 (got %d)", dim);
    ANN_SUPPORTED(p.group != 8 || dim <= 128, "group 8 supports dim <= 128 (got %d)", dim);
    FilterShape f{};
    s = search_filter(p, n, f);
    if (s != ANN_OK) return s;
    const size_t lds = (size_t)(p.waves_per_query > 1 ? 1 : p.waves_per_block) *
                       wave_lds_bytes(p.pool_cap, f, p.fp64 != 0, dim);
    ANN_SUPPORTED(lds <= (size_t)device_lds_bytes(),
                  "search plan needs %zu B of LDS per workgroup (the CU has %d)", lds,
                  device_lds_bytes());
    return ANN_OK;
}

}  // namespace ann

extern "C" size_t ann_search_plan_lds(const ann_search_plan *plan, int64_t n, int32_t dim)
{
    if (!plan || validate_plan(*plan) != ANN_OK || n < 1 || dim < 1) return 0;
    return search_wave_lds(*plan, n, dim);
}

extern "C" ann_status ann_search(const float *base, int64_t n, int32_t dim, const int32_t *graph,
                                 int32_t R, const float *queries, int32_t nq,
                                 const int32_t *entry_ids, int32_t medoid, const int32_t *k,
                                 const int32_t *L, int32_t k_max, int32_t *out_ids,
                                 float *out_dist, int32_t *stats, int32_t *trace,
                                 int32_t trace_cap, const ann_search_plan *plan, void *workspace,
                                 size_t ws_bytes, void *stream)
{
    ann_search_plan p{};
    ann_status s = search_check(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L,
                                k_max, out_ids, out_dist, trace, trace_cap, plan, workspace,
                                ws_bytes, p);
    if (s != ANN_OK) return s;
    if (nq == 0) return ANN_OK;
    return search_launch(base, n, dim, graph, R, queries, nq, entry_ids, medoid, k, L, k_max,
                         out_ids, out_dist, stats, trace, trace_cap, p,
                         static_cast<uint32_t *>(workspace), static_cast<hipStream_t>(stream),
                         true);
}
