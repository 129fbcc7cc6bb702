// Topology features of the hub nodes (feature distillation section).
//
// The paper samples a subgraph around each hub by a guided walk and encodes
// it with a graph-embedding model; here the walk is kept and the encoder is
// replaced by 32 plain statistics of the hub, its neighbourhood and the walk
// subgraph (the list is in include/ann.h).
//
// Guided walk from hub v with max hop h, one wavefront per hub: the subgraph's
// node list doubles as the FIFO.  A dequeued node u (depth < h) samples
// x = max(2, ceil(MinDeg * deg(u) / MaxDeg)) neighbours: the ceil(x/2) nearest
// and floor(x/2) farthest by (d2, id) -- all of them when deg(u) <= x.  Every
// sampled edge counts; a sampled node not yet in the subgraph (a per-hub
// bitmap in global memory) joins it one hop deeper, while the subgraph holds
// fewer than wcap nodes.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int FW_MAX = 4096;

__device__ inline double d2_ff(const float *a, const float *b, int dim)
{
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        double t = (double)a[j] - (double)b[j];
        s += t * t;
    }
    return s;
}

__device__ inline double d2_fd(const float *a, const double *m, int dim)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        double t = (double)a[j] - m[j];
        s = s + t * t;
    }
    return s;
}

__device__ inline double wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wmin(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double wmax(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline int wsumi(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline uint64_t dkey(double v)
{
    return (uint64_t)__double_as_longlong(v);   // v >= 0: bit order = value order
}

// ascending bitonic sort of one (key, id) per lane
__device__ inline void wsort(uint64_t &k, uint32_t &id)
{
    const int lane = __lane_id();
    for (int size = 2; size <= 64; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            uint64_t ok = __shfl_xor(k, stride);
            uint32_t oi = __shfl_xor(id, stride);
            bool up = (lane & size) == 0, lower = (lane & stride) == 0;
            bool mine = k < ok || (k == ok && id < oi);
            bool keep = (lower == up) ? mine : !mine;
            if (!keep) {
                k = ok;
                id = oi;
            }
        }
}

// ---- global statistics
__global__ void degree_kernel(const int32_t *graph, int64_t n, int R, int32_t *deg,
                              int32_t *indeg, int32_t *mm, unsigned long long *edges)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int c = 0;
        for (int s = 0; s < R; ++s) {
            int32_t w = graph[v * R + s];
            if (w < 0) continue;
            ++c;
            atomicAdd(&indeg[w], 1);
        }
        deg[v] = c;
        if (c > 0) {
            atomicMin(&mm[0], c);
            atomicMax(&mm[1], c);
        }
        atomicAdd(edges, (unsigned long long)c);
    }
}

__global__ void nu_partial_kernel(const float *base, int64_t n, int dim, const int32_t *graph,
                                  int R, double *part, int *cntp)
{
    __shared__ double sh[256];
    __shared__ int shc[256];
    double s = 0.0;
    int c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int32_t first = -1;
        for (int q = 0; q < R && first < 0; ++q) first = graph[v * R + q];
        if (first < 0) continue;
        s += sqrt(d2_ff(base + v * dim, base + (int64_t)first * dim, dim));
        ++c;
    }
    sh[threadIdx.x] = s;
    shc[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            shc[threadIdx.x] += shc[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sh[0];
        cntp[blockIdx.x] = shc[0];
    }
}

__global__ void csize_kernel(const int32_t *assign, int64_t n, int32_t *csize)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&csize[assign[v]], 1);
}

__global__ void zero_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

struct FeatArgs {
    const float *base;
    int64_t n;
    int dim;
    const int32_t *graph;
    int R;
    int medoid;
    const int32_t *hub_ids;
    int nh;
    const int32_t *assign;
    const double *centroids;
    int h;
    int wcap;
    const int32_t *deg;
    const int32_t *indeg;
    const int32_t *mm;
    const unsigned long long *edges;
    const double *nu_part;
    const int *nu_cnt;
    int nu_blocks;
    const int32_t *csize;
    uint32_t *bits;       // nh x words
    int64_t words;
    double *raw;          // nh x 32
    int32_t *walk_sizes;  // nh x 6 or null
};

__global__ void __launch_bounds__(64) walk_kernel(FeatArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    int32_t *S = reinterpret_cast<int32_t *>(lds);
    uint8_t *depth = reinterpret_cast<uint8_t *>(S + a.wcap);
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    uint32_t *bits = a.bits + (int64_t)c * a.words;
    // global scalars
    double nu_s = 0.0;
    int nu_c = 0;
    for (int b = 0; b < a.nu_blocks; ++b) {
        nu_s += a.nu_part[b];
        nu_c += a.nu_cnt[b];
    }
    const double nu = nu_s / (double)nu_c;
    const double mean_in = (double)(*a.edges) / (double)a.n;
    const int mindeg = a.mm[0], maxdeg = a.mm[1];
    const int32_t v = a.hub_ids[c];
    const float *xv = a.base + (int64_t)v * a.dim;

    if (lane == 0) {
        S[0] = v;
        depth[0] = 0;
        atomicOr(&bits[v >> 5], 1u << (v & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int ns = 1;
    long long wedges = 0;
    double wlen = 0.0;
    for (int head = 0; head < ns; ++head) {
        const int du_depth = depth[head];
        if (du_depth >= a.h) continue;
        const int32_t u = S[head];
        int32_t w = lane < a.R ? a.graph[(int64_t)u * a.R + lane] : -1;
        uint64_t k = ~0ull;
        uint32_t id = 0xFFFFFFFFu;
        if (w >= 0) {
            k = dkey(d2_ff(a.base + (int64_t)u * a.dim, a.base + (int64_t)w * a.dim, a.dim));
            id = (uint32_t)w;
        }
        const int m = __popcll(__ballot(w >= 0));
        wsort(k, id);
        int x = (int)(((long long)mindeg * m + maxdeg - 1) / maxdeg);
        if (x < 2) x = 2;
        const int lo_n = m <= x ? m : (x + 1) / 2;
        const int hi_n = m <= x ? 0 : x / 2;
        const bool chosen = lane < m && (lane < lo_n || lane >= m - hi_n);
        const uint64_t cb = __ballot(chosen);
        wedges += __popcll(cb);
        wlen += wsum(chosen ? sqrt(__longlong_as_double((long long)k)) : 0.0);
        bool fresh = false;
        if (chosen) {
            uint32_t bit = 1u << (id & 31u);
            fresh = (atomicOr(&bits[id >> 5], bit) & bit) == 0;
        }
        const uint64_t fb = __ballot(fresh);
        if (fresh) {
            int pos = ns + __popcll(fb & ((1ull << lane) - 1ull));
            if (pos < a.wcap) {
                S[pos] = (int32_t)id;
                depth[pos] = (uint8_t)(du_depth + 1);
            }
        }
        ns += __popcll(fb);
        if (ns > a.wcap) ns = a.wcap;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // ---- features
    double f[24];
    for (int t = 0; t < 24; ++t) f[t] = 0.0;
    f[0] = (double)a.deg[v] / a.R;
    f[1] = (double)a.indeg[v] / mean_in;
    int cnt_d[6] = {0, 0, 0, 0, 0, 0};
    int maxd = 0, other = 0;
    double so = 0.0, si = 0.0;
    for (int q = lane; q < ns; q += 64) {
        int dq = depth[q];
        if (dq <= 5) cnt_d[dq]++;
        if (dq > maxd) maxd = dq;
        int32_t w = S[q];
        if (q > 0 && a.assign[w] != c) other++;
        so += a.deg[w];
        si += a.indeg[w];
    }
    for (int t = 0; t < 6; ++t) cnt_d[t] = wsumi(cnt_d[t]);
    for (int o = 32; o > 0; o >>= 1) maxd = max(maxd, __shfl_xor(maxd, o));
    other = wsumi(other);
    so = wsum(so);
    si = wsum(si);
    for (int t = 1; t <= 5; ++t) f[1 + t] = log2(1.0 + cnt_d[t]);
    f[7] = log2(1.0 + (double)wedges);
    // out-neighbour distances
    {
        int32_t w = lane < a.R ? a.graph[(int64_t)v * a.R + lane] : -1;
        bool ok = w >= 0;
        double dv = ok ? sqrt(d2_ff(xv, a.base + (int64_t)w * a.dim, a.dim)) / nu : 0.0;
        int m = __popcll(__ballot(ok));
        if (m > 0) {
            double mean = wsum(dv) / m;
            double lo = wmin(ok ? dv : 1e300), hi = wmax(ok ? dv : -1e300);
            double q = wsum(ok ? (dv - mean) * (dv - mean) : 0.0);
            f[8] = mean;
            f[9] = lo;
            f[10] = hi;
            f[11] = sqrt(q / m);
        }
    }
    // walk-node distances (two passes)
    if (ns > 1) {
        double s = 0.0, lo = 1e300, hi = -1e300;
        for (int q = 1 + lane; q < ns; q += 64) {
            double dv = sqrt(d2_ff(xv, a.base + (int64_t)S[q] * a.dim, a.dim)) / nu;
            s += dv;
            lo = fmin(lo, dv);
            hi = fmax(hi, dv);
        }
        const int m = ns - 1;
        const double mean = wsum(s) / m;
        lo = wmin(lo);
        hi = wmax(hi);
        double qq = 0.0;
        for (int q = 1 + lane; q < ns; q += 64) {
            double dv = sqrt(d2_ff(xv, a.base + (int64_t)S[q] * a.dim, a.dim)) / nu;
            qq += (dv - mean) * (dv - mean);
        }
        qq = wsum(qq);
        f[12] = mean;
        f[13] = lo;
        f[14] = hi;
        f[15] = sqrt(qq / m);
    }
    f[16] = (double)a.csize[c] / ((double)a.n / a.nh);
    f[17] = sqrt(d2_fd(xv, a.centroids + (int64_t)c * a.dim, a.dim)) / nu;
    f[18] = sqrt(d2_ff(xv, a.base + (int64_t)a.medoid * a.dim, a.dim)) / nu;
    f[19] = ns > 1 ? (double)other / (ns - 1) : 0.0;
    f[20] = so / ns / a.R;
    f[21] = si / ns / mean_in;
    f[22] = wedges > 0 ? (wlen / (double)wedges) / nu : 0.0;
    f[23] = (double)maxd / a.h;
    if (lane < 32) a.raw[(int64_t)c * 32 + lane] = lane < 24 ? f[lane < 24 ? lane : 0] : 0.0;
    if (a.walk_sizes && lane < 6) a.walk_sizes[c * 6 + lane] = cnt_d[lane];
}

__global__ void standardise_kernel(const double *raw, int nh, int standardise, float *out)
{
    const int t = threadIdx.x;   // column
    if (t >= 32) return;
    if (!standardise) {
        for (int c = 0; c < nh; ++c) out[c * 32 + t] = (float)raw[c * 32 + t];
        return;
    }
    double s = 0.0;
    for (int c = 0; c < nh; ++c) s += raw[c * 32 + t];
    const double mean = s / nh;
    double q = 0.0;
    for (int c = 0; c < nh; ++c) {
        double z = raw[c * 32 + t] - mean;
        q += z * z;
    }
    const double sd = sqrt(q / nh);
    for (int c = 0; c < nh; ++c) out[c * 32 + t] = sd > 0 ? (float)((raw[c * 32 + t] - mean) / sd) : 0.f;
}

inline int gridn(int64_t n) { return (int)((n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256); }

constexpr int NU_BLOCKS = 1024;

}  // namespace

size_t hub_features_ws(int64_t n, int nh)
{
    int64_t words = (n + 31) / 32;
    size_t b = round_up((size_t)n * 4, 256) * 2 + round_up(64, 256) * 2;
    b += round_up(NU_BLOCKS * 8, 256) + round_up(NU_BLOCKS * 4, 256);
    b += round_up((size_t)nh * 4, 256) + round_up((size_t)nh * words * 4, 256);
    b += round_up((size_t)nh * 32 * 8, 256);
    return b;
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_hub_features(const float *base, int64_t n, int32_t dim,
                                       const int32_t *graph, int32_t R, int32_t medoid,
                                       const int32_t *hub_ids, int32_t n_hubs,
                                       const int32_t *assign, const double *centroids, int32_t h,
                                       int32_t wcap, int32_t standardise, float *features,
                                       int32_t *walk_sizes, void *workspace, size_t ws_bytes,
                                       void *stream)
{
    ANN_REQUIRE(base && graph && hub_ids && assign && centroids && features && workspace,
                "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF && dim >= 1, "bad n or dim");
    ANN_REQUIRE(R >= 1 && R <= 64, "R must be in [1, 64]");
    ANN_REQUIRE(medoid >= 0 && medoid < n, "medoid out of range");
    ANN_REQUIRE(n_hubs >= 1 && n_hubs <= n, "n_hubs must be in [1, n]");
    ANN_REQUIRE(h >= 1 && h <= 250, "h must be in [1, 250]");
    ANN_REQUIRE(wcap >= 1 && wcap <= FW_MAX, "wcap must be in [1, 4096]");
    ANN_REQUIRE(ws_bytes >= ann_workspace_size(ANN_OP_HUB_FEATURES, n, dim, n_hubs, R),
                "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    int32_t *deg = cv.take<int32_t>((size_t)n);
    int32_t *indeg = cv.take<int32_t>((size_t)n);
    int32_t *mm = cv.take<int32_t>(16);
    unsigned long long *edges = cv.take<unsigned long long>(8);
    double *nu_part = cv.take<double>(NU_BLOCKS);
    int *nu_cnt = cv.take<int>(NU_BLOCKS);
    int32_t *csize = cv.take<int32_t>((size_t)n_hubs);
    const int64_t words = (n + 31) / 32;
    uint32_t *bits = cv.take<uint32_t>((size_t)n_hubs * words);
    double *raw = cv.take<double>((size_t)n_hubs * 32);

    hipLaunchKernelGGL(zero_u32, dim3(gridn(n)), dim3(256), 0, st, (uint32_t *)indeg, n);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(zero_u32, dim3(gridn(n_hubs)), dim3(256), 0, st, (uint32_t *)csize,
                       (int64_t)n_hubs);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(zero_u32, dim3(gridn((int64_t)n_hubs * words)), dim3(256), 0, st, bits,
                       (int64_t)n_hubs * words);
    ANN_LAUNCHED();
    int32_t mm_init[2] = {0x7fffffff, 0};
    unsigned long long e0 = 0;
    ANN_HIP(hipMemcpyAsync(mm, mm_init, sizeof(mm_init), hipMemcpyHostToDevice, st));
    ANN_HIP(hipMemcpyAsync(edges, &e0, sizeof(e0), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(degree_kernel, dim3(gridn(n)), dim3(256), 0, st, graph, n, R, deg, indeg, mm,
                       edges);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(nu_partial_kernel, dim3(NU_BLOCKS), dim3(256), 0, st, base, n, dim, graph, R,
                       nu_part, nu_cnt);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(csize_kernel, dim3(gridn(n)), dim3(256), 0, st, assign, n, csize);
    ANN_LAUNCHED();
    FeatArgs a{};
    a.base = base;
    a.n = n;
    a.dim = dim;
    a.graph = graph;
    a.R = R;
    a.medoid = medoid;
    a.hub_ids = hub_ids;
    a.nh = n_hubs;
    a.assign = assign;
    a.centroids = centroids;
    a.h = h;
    a.wcap = wcap;
    a.deg = deg;
    a.indeg = indeg;
    a.mm = mm;
    a.edges = edges;
    a.nu_part = nu_part;
    a.nu_cnt = nu_cnt;
    a.nu_blocks = NU_BLOCKS;
    a.csize = csize;
    a.bits = bits;
    a.words = words;
    a.raw = raw;
    a.walk_sizes = walk_sizes;
    size_t lds = round_up((size_t)wcap * 5, 16);
    hipLaunchKernelGGL(walk_kernel, dim3(n_hubs), dim3(64), lds, st, a);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(standardise_kernel, dim3(1), dim3(64), 0, st, raw, n_hubs, standardise,
                       features);
    ANN_LAUNCHED();
    return ANN_OK;
}
