// The entry stage's search over the hub navigation graph (high-tier graph
// section: Algorithm 1 run on the hub graph), specialised for what that
// graph is: small (at most 2^16 hubs, an exact visited bitset fits in a few
// hundred bytes of LDS), narrow beams (L <= 64, so the whole pool lives in
// the wavefront's registers, one entry per lane) and short unit embeddings
// (dim <= 256, four lanes per vector).
//
// One wavefront per query.  A pool entry is the 64-bit word (FP32 distance
// bits << 32 | hub index), bit 31 marking "expanded": distances are
// non-negative, so with that bit masked the word order is the (distance,
// index) order.  Each step expands the first unexpanded entry (a ballot),
// tests its neighbours against the visited bitset in slot order, computes the
// new neighbours' squared distances (four lanes per vector, two shuffle
// steps) and merges them into the pool at once: the keys that can enter
// (all while the pool has room, else those below its last entry) are passed
// over once, which gives every pool entry the number of them below it and
// each of them the number of pool entries and of kept keys below it; each
// word is written to its merged place in LDS and the first L places are read
// back.  Keeping
// the L smallest of pool and new keys is what inserting them one at a time
// (when the pool has room or the key beats its last entry) keeps, so this is
// the bounded best-first search of ann_search with k = 1 and an exact visited
// set.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr uint64_t kEmpty64 = ~0ull;
constexpr uint64_t kExp = 1ull << 31;           // "expanded", in the index half of a word
constexpr uint64_t kKeyMask = ~kExp;
constexpr int kQuadSwap1 = 0xB1;   // DPP quad permutation [1, 0, 3, 2]
constexpr int kQuadSwap2 = 0x4E;   // DPP quad permutation [2, 3, 0, 1]

__device__ inline uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// v with lane l replaced by the wave-uniform value x: one v_writelane_b32
// (clang exposes no builtin for it here), its lane select in M0, since a
// VALU instruction reads at most one SGPR on this target; M0 is a reserved
// register, so its value is kept in an SGPR of the statement's own and put back
__device__ inline int writelane(int v, int x, int l)
{
    int keep;
    asm("s_mov_b32 %1, m0\n\ts_mov_b32 m0, %3\n\tv_writelane_b32 %0, %2, m0\n\ts_mov_b32 m0, %1"
        : "+v"(v), "=&s"(keep)
        : "s"(x), "s"(l));
    return v;
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

// LDS of one wavefront: 64 merge words, 64 staged ids, the visited bitset
// (a multiple of 16 bytes, so that every wavefront's words stay aligned)
__host__ __device__ inline size_t hub_wave_lds(int vis_words)
{
    return ((size_t)64 * 8 + 64 * 4 + (size_t)vis_words * 4 + 15) / 16 * 16;
}

// T = float4 chunks per lane of a vector (the vector's dim / 16, rounded up);
// FULL: the dim is exactly 16 T, so every lane's chunks are inside the vector
template <int T, bool FULL>
__global__ void __launch_bounds__(256) hub_search_kernel(HubArgs a)
{
    extern __shared__ __align__(16) unsigned char hs_lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qi = blockIdx.x * 4 + wave;
    if (qi >= a.nq) return;                       // whole wavefront
    unsigned char *wl = hs_lds + (size_t)wave * hub_wave_lds(a.vis_words);
    uint64_t *merged = reinterpret_cast<uint64_t *>(wl);              // 64 words
    int32_t *stage = reinterpret_cast<int32_t *>(wl + 64 * 8);         // 64 ids
    uint32_t *vis = reinterpret_cast<uint32_t *>(wl + 64 * 8 + 64 * 4);
    for (int w = lane; w < a.vis_words; w += 64) vis[w] = 0u;
    const int chunks = a.dim >> 2;
    const int gl = lane & 3, grp = lane >> 2;
    const float4 *e4 = reinterpret_cast<const float4 *>(a.emb);
    float4 q[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int ch = gl + 4 * t;
        q[t] = FULL || ch < chunks
                   ? reinterpret_cast<const float4 *>(a.qemb)[(size_t)qi * chunks + ch]
                   : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // squared distance of hub `id` (valid in the four lanes of the group):
    // all of a lane's chunks are requested before any is used (a chunk past
    // the vector's end re-reads chunk 0 and adds nothing), and the group's
    // four partial sums meet through two DPP quad permutations
    auto dist = [&](int id) {
        float4 x[T];
        // id < 2^16 and chunks <= 64: the row offset is a 24-bit product
        const float4 *row = e4 + (size_t)__umul24((unsigned)id, (unsigned)chunks);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int ch = gl + 4 * t;
            x[t] = row[FULL || ch < chunks ? ch : 0];
        }
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float dx = x[t].x - q[t].x, dy = x[t].y - q[t].y, dz = x[t].z - q[t].z,
                        dw = x[t].w - q[t].w;
            const float part = dx * dx + dy * dy + dz * dz + dw * dw;
            acc += FULL || gl + 4 * t < chunks ? part : 0.f;
        }
        acc += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), kQuadSwap1,
                                                          0xf, 0xf, false));
        acc += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc), kQuadSwap2,
                                                          0xf, 0xf, false));
        return acc;
    };
    int32_t *tr = a.trace ? a.trace + (size_t)qi * a.trace_cap : nullptr;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // the entry
    uint64_t P = kEmpty64;
    {
        const float d = dist(a.start);
        if (lane == 0) {
            P = ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)a.start;
            vis[a.start >> 5] = 1u << (a.start & 31);
        }
    }
    int cnt = 1, ndc = 1, hops = 0;
    // the adjacency row of the old pool's next unexpanded entry, requested
    // one step ahead; used only when that entry is the node expanded next
    int pre_node = -1;
    int32_t pre_nb = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (;;) {
        // lanes at or beyond cnt hold kEmpty64, whose expanded bit is set
        const uint64_t un = __ballot(!(P & kExp));
        if (!un) break;
        const int pl = __ffsll((unsigned long long)un) - 1;
        const int p = (int)((uint32_t)readlane64(P, pl) & 0xffffu);
        if (lane == pl) P |= kExp;
        if (tr && lane == 0 && hops < a.trace_cap) tr[hops] = p;
        ++hops;
        const int32_t nb = p == pre_node ? pre_nb
                                         : (lane < a.s ? a.graph[(size_t)p * a.s + lane] : -1);
        // the word's old bits come out of the branch, not a flag, so that the
        // test below is one compare mask
        const bool inb = nb >= 0 && nb < a.n_hubs;
        const uint32_t bit = 1u << (nb & 31);
        uint32_t old = bit;
        if (inb) old = atomicOr(&vis[nb >> 5], bit);
        const bool fresh = !(old & bit);
        // requested after the expanded row has been consumed, so that no
        // wait for that row also waits for this one
        const uint64_t un2 = un & (un - 1);
        pre_node = un2 ? (int)((uint32_t)readlane64(P, __ffsll((unsigned long long)un2) - 1) &
                               0xffffu)
                       : -1;
        if (pre_node >= 0) pre_nb = lane < a.s ? a.graph[(size_t)pre_node * a.s + lane] : -1;
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
            // the new keys that can enter: all while the pool has room, else
            // those below its last entry (the others would be dropped by the
            // merge anyway)
            bool keep = (lane & 3) == 0 && (lane >> 2) < nb_batch;
            if (cnt == a.L) keep = keep && key < (readlane64(P, a.L - 1) & kKeyMask);
            const uint64_t km = __ballot(keep);
            if (!km) continue;
            const int nkeep = __popcll(km);
            // merge: the pool entry in lane j goes to j + (kept keys below
            // it); a kept key to (pool entries below it) + (kept keys below
            // it).  Keys are distinct (distinct indices), so "not below" is
            // "above".  An empty lane's word (kEmpty64 with the expanded bit
            // cleared) is above every key, so the pool entries below a key
            // are the lanes whose word is not above it.
            const uint64_t pk = P & kKeyMask;
            int up = 0, below = 0, rank = 0;
            for (uint64_t mm = km; mm; mm &= mm - 1) {
                const int l = __ffsll((unsigned long long)mm) - 1;
                const uint64_t nk = readlane64(key, l);
                const bool lt = nk < pk;
                up += lt ? 1 : 0;
                below = writelane(below, __popcll(~__ballot(lt)), l);
                rank += nk < key ? 1 : 0;
            }
            const int ncnt = cnt + nkeep < a.L ? cnt + nkeep : a.L;
            __builtin_amdgcn_wave_barrier();      // the last merge's reads of `merged` are done
            if (lane < cnt && lane + up < ncnt) merged[lane + up] = P;
            if (keep && below + rank < ncnt) merged[below + rank] = key;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            P = lane < ncnt ? merged[lane] : kEmpty64;
            cnt = ncnt;
        }
    }
    if (lane == 0) {
        a.best[qi] = (int32_t)((uint32_t)P & 0xffffu);
        a.best_d2[qi] = __uint_as_float((uint32_t)(P >> 32));
        if (a.stats) {
            a.stats[2 * qi] = ndc;
            a.stats[2 * qi + 1] = hops;
        }
    }
    if (tr)
        for (int t = hops + lane; t < a.trace_cap; t += 64) tr[t] = -1;
}

template <int T>
void launch_hub(const HubArgs &a, dim3 grid, size_t lds, hipStream_t st)
{
    if (a.dim / 4 == 4 * T)
        hipLaunchKernelGGL((hub_search_kernel<T, true>), grid, dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((hub_search_kernel<T, false>), grid, dim3(256), lds, st, a);
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
    const size_t lds = 4 * hub_wave_lds(a.vis_words);
    const dim3 grid((unsigned)((nq + 3) / 4));
    const int T = (dim / 4 + 3) / 4;
    if (T <= 1) launch_hub<1>(a, grid, lds, st);
    else if (T <= 2) launch_hub<2>(a, grid, lds, st);
    else if (T <= 4) launch_hub<4>(a, grid, lds, st);
    else if (T <= 8) launch_hub<8>(a, grid, lds, st);
    else launch_hub<16>(a, grid, lds, st);
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
