// The entry stage's search over the hub navigation graph (high-tier graph
// section: Algorithm 1 run on the hub graph), specialised for what that
// graph is: small (at most 2^16 hubs, an exact visited bitset fits in a few
// hundred bytes of LDS), narrow beams (L <= 64, so the whole pool lives in
// the wavefront's registers, one entry per lane) and short unit embeddings
// (dim <= 256, four lanes per vector).
//
// One wavefront per query.  A pool entry is the 64-bit word (FP32 distance
// bits << 32 | hub index): distances are non-negative, so the word order is
// the (distance, index) order.  Each step expands the first unexpanded entry
// (a ballot), tests its neighbours against the visited bitset in slot order,
// computes the new neighbours' squared distances (four lanes per vector, two
// shuffle steps) and inserts them one at a time in slot order, each where
// the ballot of smaller pool entries puts it, if the pool has room or it
// beats the last entry: the bounded best-first search of ann_search with
// k = 1 and an exact visited set, without any LDS traffic for the pool.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr uint64_t kEmpty64 = ~0ull;

__device__ inline uint64_t shfl_up1(uint64_t v)
{
    const int lo = __shfl_up((int)(uint32_t)v, 1);
    const int hi = __shfl_up((int)(uint32_t)(v >> 32), 1);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ inline uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

struct HubArgs {
    const float *emb;
    int n_hubs;
    int dim;
    const int32_t *graph;
    int s;
    const float *qemb;
    int nq;
    int start;
    int L;
    int32_t *best;
    float *best_d2;
    int32_t *stats;
    int32_t *trace;
    int trace_cap;
    int vis_words;   // bitset words per wavefront
};

// T = float4 chunks per lane of a vector (the vector's dim / 16, rounded up)
template <int T>
__global__ void __launch_bounds__(256) hub_search_kernel(HubArgs a)
{
    extern __shared__ __align__(16) unsigned char hs_lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qi = blockIdx.x * 4 + wave;
    if (qi >= a.nq) return;                       // whole wavefront
    uint32_t *vis = reinterpret_cast<uint32_t *>(hs_lds) + (size_t)wave * (a.vis_words + 64);
    int32_t *stage = reinterpret_cast<int32_t *>(vis + a.vis_words);
    for (int w = lane; w < a.vis_words; w += 64) vis[w] = 0u;
    const int chunks = a.dim >> 2;
    const int gl = lane & 3, grp = lane >> 2;
    const float4 *e4 = reinterpret_cast<const float4 *>(a.emb);
    float4 q[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int ch = gl + 4 * t;
        q[t] = ch < chunks ? reinterpret_cast<const float4 *>(a.qemb)[(size_t)qi * chunks + ch]
                           : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // squared distance of hub `id` (valid in the four lanes of the group)
    auto dist = [&](int id) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int ch = gl + 4 * t;
            if (ch < chunks) {
                const float4 x = e4[(size_t)id * chunks + ch];
                const float dx = x.x - q[t].x, dy = x.y - q[t].y, dz = x.z - q[t].z,
                            dw = x.w - q[t].w;
                acc += dx * dx + dy * dy + dz * dz + dw * dw;
            }
        }
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        return acc;
    };
    int32_t *tr = a.trace ? a.trace + (size_t)qi * a.trace_cap : nullptr;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // the entry
    uint64_t P = kEmpty64;
    bool ex = false;
    {
        const float d = dist(a.start);
        if (lane == 0) {
            P = ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)a.start;
            vis[a.start >> 5] = 1u << (a.start & 31);
        }
    }
    int cnt = 1, ndc = 1, hops = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (;;) {
        const uint64_t un = __ballot(lane < cnt && !ex);
        if (!un) break;
        const int pl = __ffsll((unsigned long long)un) - 1;
        const int p = (int)(uint32_t)readlane64(P, pl);
        if (lane == pl) ex = true;
        if (tr && lane == 0 && hops < a.trace_cap) tr[hops] = p;
        ++hops;
        const int32_t nb = lane < a.s ? a.graph[(size_t)p * a.s + lane] : -1;
        bool fresh = false;
        if (nb >= 0 && nb < a.n_hubs) {
            const uint32_t bit = 1u << (nb & 31);
            fresh = !(atomicOr(&vis[nb >> 5], bit) & bit);
        }
        const uint64_t fb = __ballot(fresh);
        const int m = __popcll(fb);
        if (m == 0) continue;
        __builtin_amdgcn_wave_barrier();          // the last step's reads of stage are done
        if (fresh)
            stage[__builtin_amdgcn_mbcnt_hi((uint32_t)(fb >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)fb, 0u))] = nb;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        ndc += m;
        for (int b0 = 0; b0 < m; b0 += 16) {
            const int c = b0 + grp;
            const int id = c < m ? stage[c] : a.start;
            const float d = dist(id);
            const uint64_t key = ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)id;
            const int nb_batch = m - b0 < 16 ? m - b0 : 16;
            // insert in slot order, one at a time
            for (int g = 0; g < nb_batch; ++g) {
                const uint64_t nk = readlane64(key, 4 * g);
                if (cnt == a.L &&
                    nk >= readlane64(P, __builtin_amdgcn_readfirstlane(cnt) - 1))
                    continue;
                const int pos = __popcll(__ballot(lane < cnt && P < nk));
                const uint64_t Pu = shfl_up1(P);
                const bool eu = __shfl_up((int)ex, 1) != 0;
                if (lane > pos) {
                    P = Pu;
                    ex = eu;
                } else if (lane == pos) {
                    P = nk;
                    ex = false;
                }
                cnt = cnt < a.L ? cnt + 1 : a.L;
            }
        }
    }
    if (lane == 0) {
        a.best[qi] = (int32_t)(uint32_t)P;
        a.best_d2[qi] = __uint_as_float((uint32_t)(P >> 32));
        if (a.stats) {
            a.stats[2 * qi] = ndc;
            a.stats[2 * qi + 1] = hops;
        }
    }
    if (tr)
        for (int t = hops + lane; t < a.trace_cap; t += 64) tr[t] = -1;
}

}  // namespace

bool hub_search_supported(int n_hubs, int dim, int s, int L)
{
    return n_hubs >= 1 && n_hubs <= (1 << 16) && dim >= 4 && dim % 4 == 0 && dim <= 256 &&
           s >= 1 && s <= 64 && L >= 1 && L <= 64;
}

ann_status hub_search_launch(const float *emb, int n_hubs, int dim, const int32_t *graph, int s,
                             const float *qemb, int nq, int start, int L, int32_t *best,
                             float *best_d2, int32_t *stats, int32_t *trace, int trace_cap,
                             hipStream_t st)
{
    HubArgs a{emb, n_hubs, dim, graph, s, qemb, nq, start, L, best, best_d2, stats,
              trace, trace ? trace_cap : 0, (n_hubs + 31) / 32};
    const size_t lds = (size_t)4 * (a.vis_words + 64) * 4;
    const dim3 grid((unsigned)((nq + 3) / 4));
    const int T = (dim / 4 + 3) / 4;
    if (T <= 1) hipLaunchKernelGGL(hub_search_kernel<1>, grid, dim3(256), lds, st, a);
    else if (T <= 2) hipLaunchKernelGGL(hub_search_kernel<2>, grid, dim3(256), lds, st, a);
    else if (T <= 4) hipLaunchKernelGGL(hub_search_kernel<4>, grid, dim3(256), lds, st, a);
    else if (T <= 8) hipLaunchKernelGGL(hub_search_kernel<8>, grid, dim3(256), lds, st, a);
    else hipLaunchKernelGGL(hub_search_kernel<16>, grid, dim3(256), lds, st, a);
    ANN_LAUNCHED();
    return ANN_OK;
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_hub_search(const float *emb, int32_t n_hubs, int32_t dim,
                                     const int32_t *graph, int32_t s, const float *qemb, int32_t nq,
                                     int32_t start, int32_t L, int32_t *best, float *best_d2,
                                     int32_t *stats, int32_t *trace, int32_t trace_cap,
                                     void *stream)
{
    ANN_REQUIRE(nq >= 0, "nq must be >= 0");
    ANN_REQUIRE(emb && graph && (nq == 0 || (qemb && best && best_d2)), "a required pointer is NULL");
    ANN_SUPPORTED(hub_search_supported(n_hubs, dim, s, L),
                  "hub search needs 1 <= n_hubs <= 65536, dim % 4 == 0 and 4 <= dim <= 256, "
                  "1 <= s <= 64, 1 <= L <= 64 (got %d, %d, %d, %d)", n_hubs, dim, s, L);
    ANN_REQUIRE(start >= 0 && start < n_hubs, "start out of range");
    ANN_REQUIRE(aligned(emb, 16) && aligned(qemb, 16), "emb/qemb must be 16-byte aligned");
    ANN_REQUIRE(trace == nullptr || trace_cap >= 1, "trace_cap must be >= 1 with a trace buffer");
    if (nq == 0) return ANN_OK;
    return hub_search_launch(emb, n_hubs, dim, graph, s, qemb, nq, start, L, best, best_d2, stats,
                             trace, trace_cap, static_cast<hipStream_t>(stream));
}
