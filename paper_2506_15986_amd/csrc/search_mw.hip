// Batched best-first beam search with several wavefronts per query: one
// workgroup of W = 2 or 4 wavefronts serves one query at a time (persistent
// grid, atomic work counter).  Wave 0 runs the pool, the visited filter and
// the merge; all W waves gather and reduce the new neighbours' distances, so
// W times as many vectors are in flight per hop.  Worth it for wide vectors,
// where one wavefront holds only a few vectors in registers.  Results are
// those of the single-wavefront kernel with the same gather group (each
// distance is summed by one lane group in the same order).  FP32, gather
// group 16.
#include "beam.h"
#include "common.h"
#include "internal.h"
#include "search_core.h"

namespace ann {
namespace {

using namespace beam;

template <int CPL, int FILT, int W>
__global__ void __launch_bounds__(256) search_mw_kernel(SearchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int ctrl[2];
    using S = Searcher<16, CPL, false, FILT>;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    S s;
    s.setup(smem, a.pool_cap, a.visited_log2, a.filter, a.n, a.base, a.dim, a.graph, a.R);
    for (;;) {
        if (threadIdx.x == 0) ctrl[1] = (int)atomicAdd(a.counter, 1u);
        __syncthreads();
        const int slot = __builtin_amdgcn_readfirstlane(((volatile int *)ctrl)[1]);
        __syncthreads();
        if (slot >= a.nq) break;
        const int qi = a.order ? a.order[slot] : slot;
        if (qi < 0 || qi >= a.nq) continue;
        const int kq = a.k[qi];
        const int Lq = a.L[qi];
        const int entry = a.entry ? a.entry[qi] : a.medoid;
        int32_t *trace = a.trace ? a.trace + (size_t)qi * a.trace_cap : nullptr;
        if (kq < 1 || kq > Lq || Lq > a.pool_cap || kq > a.k_max || entry < 0 ||
            (int64_t)entry >= a.n) {
            if (w == 0) {
                int32_t *oid = a.out_ids + (size_t)qi * a.k_max;
                float *odist = a.out_dist + (size_t)qi * a.k_max;
                for (int t = lane; t < a.k_max; t += 64) {
                    oid[t] = -1;
                    odist[t] = __int_as_float(0x7f800000);
                }
                for (int t = lane; trace && t < a.trace_cap; t += 64) trace[t] = -1;
                if (a.stats && lane == 0) {
                    int32_t *st = a.stats + (size_t)qi * 4;
                    st[0] = 0; st[1] = 0; st[2] = 0; st[3] = 2;
                }
            }
            continue;
        }
        if (w == 0) s.load_query(a.queries + (size_t)qi * a.dim);
        __syncthreads();
        SearchResult r = s.template run_multi<W>((uint32_t)entry, Lq, trace, a.trace_cap, w, ctrl);
        if (w == 0) {
            int32_t *oid = a.out_ids + (size_t)qi * a.k_max;
            float *odist = a.out_dist + (size_t)qi * a.k_max;
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
}

template <int CPL, int FILT, int W>
ann_status launch_mw(const SearchArgs &a, int blocks, hipStream_t st)
{
    auto kern = search_mw_kernel<CPL, FILT, W>;
    const size_t lds = a.wave_lds;
    if (lds > 65536) ANN_HIP(hipFuncSetAttribute((const void *)kern,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds));
    if (blocks <= 0) {
        int per_cu = 0;
        ANN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * W, lds));
        if (per_cu < 1) return fail(ANN_ENOTSUP, "search plan does not fit on a CU (%zu B LDS)", lds);
        blocks = per_cu * device_cus();
    }
    if (blocks > a.nq) blocks = a.nq;
    if (blocks < 1) blocks = 1;
    if (!a.order) {   // with the query-order pre-pass its sort kernel zeroed it
        ann_status rs = reset_work_counter(a.counter, st);
        if (rs != ANN_OK) return rs;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * W), lds, st, a);
    ANN_LAUNCHED();
    return ANN_OK;
}

template <int CPL, int W>
ann_status by_filter(const SearchArgs &a, int blocks, hipStream_t st)
{
    switch (a.filter.kind) {
    case kBitset: return launch_mw<CPL, kBitset, W>(a, blocks, st);
    case kTag16: return launch_mw<CPL, kTag16, W>(a, blocks, st);
    case kTag12: return launch_mw<CPL, kTag12, W>(a, blocks, st);
    case kId32: return launch_mw<CPL, kId32, W>(a, blocks, st);
    default: break;
    }
    return fail(ANN_ENOTSUP, "unknown filter form %d", a.filter.kind);
}

template <int W>
ann_status by_chunks(const SearchArgs &a, int blocks, hipStream_t st)
{
    const int cpl = (a.dim / 4 + 15) / 16;
    if (cpl <= 1) return by_filter<1, W>(a, blocks, st);
    if (cpl <= 2) return by_filter<2, W>(a, blocks, st);
    if (cpl <= 4) return by_filter<4, W>(a, blocks, st);
    if (cpl <= 8) return by_filter<8, W>(a, blocks, st);
    if (cpl <= 15) return by_filter<15, W>(a, blocks, st);
    if (cpl <= 16) return by_filter<16, W>(a, blocks, st);
    return fail(ANN_ENOTSUP, "dim %d exceeds 1024", a.dim);
}

}  // namespace

ann_status launch_search_mw(const SearchArgs &a, int waves_per_query, int blocks, hipStream_t st)
{
    if (waves_per_query == 2) return by_chunks<2>(a, blocks, st);
    if (waves_per_query == 4) return by_chunks<4>(a, blocks, st);
    return fail(ANN_ENOTSUP, "waves_per_query %d", waves_per_query);
}

}  // namespace ann
