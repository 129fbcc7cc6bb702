// Candidate lists for the NSG-style graph: the union, per point, of two id
// lists (the pool of a search for the point itself and its exact kNN list),
// with the point's own id and repeats dropped, ordered by (squared L2, id).
//
// One workgroup of 256 threads per point.  The ids go to LDS; eight lanes
// form each FP64 squared distance (lane j of the eight sums dimensions
// j, j+8, ...; the eight partial sums are combined by a butterfly, the order
// of the pruning kernel).  The (distance bits, id) pairs are sorted by a
// bitonic network in LDS; equal ids then sit next to each other, so the first
// of each run survives.  A prefix count places the survivors.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int MT = 256;
constexpr int MPG = 8;              // lanes per distance
constexpr int MERGE_MAX = 1024;     // widest union

__device__ inline bool pair_less(uint64_t ka, int32_t ia, uint64_t kb, int32_t ib)
{
    return ka < kb || (ka == kb && (uint32_t)ia < (uint32_t)ib);
}

__global__ void merge_flag_clear_kernel(int32_t *flag) { *flag = 0; }

__global__ void __launch_bounds__(MT) merge_kernel(const float *base, int64_t n, int dim,
                                                   const int32_t *a, int aw, const int32_t *b,
                                                   int bw, int P, int32_t *out_ids,
                                                   double *out_d2, int32_t *bad)
{
    extern __shared__ unsigned char smem[];
    uint64_t *key = reinterpret_cast<uint64_t *>(smem);
    int32_t *id = reinterpret_cast<int32_t *>(key + P);
    int32_t *cnt = id + P;   // MT + 1 entries
    const int64_t p = blockIdx.x;
    const int W = aw + bw;
    const int t = threadIdx.x;

    int badl = 0;
    for (int e = t; e < P; e += MT) {
        int32_t c = -1;
        if (e < aw)
            c = a[p * aw + e];
        else if (e < W)
            c = b[p * bw + (e - aw)];
        if (c < -1 || (int64_t)c >= n) {
            badl = 1;
            c = -1;
        }
        if ((int64_t)c == p) c = -1;
        id[e] = c;
        key[e] = ~0ull;
    }
    if (badl) atomicOr(bad, 1);
    __syncthreads();

    // FP64 squared distances, eight lanes per entry
    const int gi = t / MPG, gl = t % MPG;
    const float *xp = base + p * dim;
    for (int e0 = 0; e0 < W; e0 += MT / MPG) {
        const int e = e0 + gi;
        const int32_t c = e < W ? id[e] : -1;
        double acc = 0.0;
        if (c >= 0) {
            const float *xc = base + (int64_t)c * dim;
            for (int j = gl; j < dim; j += MPG) {
                const double df = (double)xp[j] - (double)xc[j];
                acc += df * df;
            }
        }
        for (int o = MPG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (gl == 0 && c >= 0) key[e] = (uint64_t)__double_as_longlong(acc);
    }
    __syncthreads();

    // bitonic sort of the P (key, id) pairs, ascending
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = t; q < P / 2; q += MT) {
                const int lo = 2 * q - (q & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t kl = key[lo], kh = key[hi];
                const int32_t il = id[lo], ih = id[hi];
                const bool sw = up ? pair_less(kh, ih, kl, il) : pair_less(kl, il, kh, ih);
                if (sw) {
                    key[lo] = kh;
                    key[hi] = kl;
                    id[lo] = ih;
                    id[hi] = il;
                }
            }
            __syncthreads();
        }
    }

    // survivors: valid and not a repeat of the entry before
    const int chunk = P >= MT ? P / MT : 1;
    const int e_lo = t * chunk, e_hi = (e_lo + chunk < P) ? e_lo + chunk : P;
    int mine = 0;
    for (int e = e_lo; e < e_hi; ++e)
        mine += id[e] >= 0 && (e == 0 || id[e] != id[e - 1]);
    cnt[t] = mine;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int s = 0; s < MT; ++s) {
            const int v = cnt[s];
            cnt[s] = run;
            run += v;
        }
        cnt[MT] = run;
    }
    __syncthreads();
    int pos = cnt[t];
    int32_t *oi = out_ids + p * W;
    double *od = out_d2 + p * W;
    for (int e = e_lo; e < e_hi; ++e) {
        if (id[e] >= 0 && (e == 0 || id[e] != id[e - 1])) {
            oi[pos] = id[e];
            od[pos] = __longlong_as_double((long long)key[e]);
            ++pos;
        }
    }
    for (int s = cnt[MT] + t; s < W; s += MT) {
        oi[s] = -1;
        od[s] = __longlong_as_double(0x7FF0000000000000ll);
    }
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" size_t ann_merge_candidates_workspace_size(void) { return 256; }

extern "C" ann_status ann_merge_candidates(const float *base, int64_t n, int32_t dim,
                                           const int32_t *a_ids, int32_t a_w,
                                           const int32_t *b_ids, int32_t b_w, int32_t *out_ids,
                                           double *out_d2, void *workspace, size_t ws_bytes,
                                           void *stream)
{
    ANN_REQUIRE(base && out_ids && out_d2 && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(a_w >= 0 && b_w >= 0, "list widths must be >= 0");
    ANN_REQUIRE(a_w + b_w >= 1 && a_w + b_w <= MERGE_MAX, "a_w + b_w must be in [1, %d]",
                MERGE_MAX);
    ANN_REQUIRE(a_w == 0 || a_ids, "a_ids is NULL");
    ANN_REQUIRE(b_w == 0 || b_ids, "b_ids is NULL");
    ANN_REQUIRE(ws_bytes >= 256, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t *bad = static_cast<int32_t *>(workspace);
    int P = 64;
    while (P < a_w + b_w) P <<= 1;
    const size_t lds = (size_t)P * (sizeof(uint64_t) + sizeof(int32_t)) + (MT + 1) * sizeof(int32_t);
    hipLaunchKernelGGL(merge_flag_clear_kernel, dim3(1), dim3(1), 0, st, bad);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)n), dim3(MT), lds, st, base, n, (int)dim, a_ids,
                       (int)a_w, b_ids, (int)b_w, P, out_ids, out_d2, bad);
    ANN_LAUNCHED();
    int32_t h = 0;
    ANN_HIP(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    ANN_REQUIRE(!h, "a candidate id lies outside [-1, n)");
    return ANN_OK;
}
