// Hub nodes (Definition 3) on Lloyd k-means clusters.
//
// Assignment: each point goes to argmin_c (d2(x, mu_c), c) where d2 is the
// FP64 sum over dimensions in order, each term (x_j - mu_cj)^2 rounded
// separately (no fused multiply-add) -- the same arithmetic as a plain
// sequential loop, so every decision is reproducible bit for bit.  A block
// stages 64 points in LDS and streams the centroids through LDS in chunks of
// 32; wavefront w of the block scores centroids 8w..8w+7 of each chunk for
// all 64 points.
// Update: per-cluster FP64 sums by atomic adds (exact when the data sit on a
// dyadic grid whose partial sums fit in 53 bits, so order does not matter),
// mean = sum / count; an empty cluster keeps its centroid.  The loop stops
// after an assignment step that changes nothing, or after `iters` steps.
// Hub of a cluster: the member nearest its mean by (d2, id); an empty
// cluster takes the nearest point that is not yet a hub (cluster order).
#include <cmath>
#include <unordered_set>
#include <vector>

#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int KP = 64;    // points per block
constexpr int KC = 32;    // centroids per LDS chunk
constexpr int KD = 128;   // dims per LDS stage

__device__ inline double term(float x, double m)
{
#pragma clang fp contract(off)
    double t = (double)x - m;
    return t * t;
}

__device__ inline double d2_to(const float *x, const double *m, int dim)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int j = 0; j < dim; ++j) s = s + term(x[j], m[j]);
    return s;
}

__global__ void __launch_bounds__(256) assign_kernel(const float *base, int64_t n, int dim,
                                                     const double *mu, int nh, int32_t *assign,
                                                     int32_t *changed)
{
#pragma clang fp contract(off)
    __shared__ float xs[KP][KD + 1];
    __shared__ double ms[KC][KD];
    __shared__ double bestv[4][KP];
    __shared__ int bestc[4][KP];
    const int t = threadIdx.x;
    const int p = t & 63;          // point within the block
    const int g = t >> 6;          // wave: centroids 8g..8g+7 of each chunk
    const int64_t i = (int64_t)blockIdx.x * KP + p;
    double bv = __longlong_as_double(0x7ff0000000000000ll);
    int bc = 0x7fffffff;
    for (int c0 = 0; c0 < nh; c0 += KC) {
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
        for (int d0 = 0; d0 < dim; d0 += KD) {
            const int dd = dim - d0 < KD ? dim - d0 : KD;
            __syncthreads();
            for (int e = t; e < KP * KD; e += 256) {
                int r = e / KD, j = e % KD;
                int64_t g2 = (int64_t)blockIdx.x * KP + r;
                xs[r][j] = (g2 < n && j < dd) ? base[g2 * dim + d0 + j] : 0.f;
            }
            for (int e = t; e < KC * KD; e += 256) {
                int r = e / KD, j = e % KD;
                ms[r][j] = (c0 + r < nh && j < dd) ? mu[(int64_t)(c0 + r) * dim + d0 + j] : 0.0;
            }
            __syncthreads();
            for (int j = 0; j < dd; ++j) {
                const float xv = xs[p][j];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[u] = acc[u] + term(xv, ms[8 * g + u][j]);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            int c = c0 + 8 * g + u;
            if (c < nh && (acc[u] < bv || (acc[u] == bv && c < bc))) {
                bv = acc[u];
                bc = c;
            }
        }
    }
    bestv[g][p] = bv;
    bestc[g][p] = bc;
    __syncthreads();
    if (g == 0 && i < n) {
        for (int q = 1; q < 4; ++q) {
            double v = bestv[q][p];
            int c = bestc[q][p];
            if (v < bv || (v == bv && c < bc)) {
                bv = v;
                bc = c;
            }
        }
        if (assign[i] != bc) {
            assign[i] = bc;
            *changed = 1;
        }
    }
}

// ---- assignment on the matrix cores, with a certified shortlist.
//
// The step above spends 3 FP64 operations per (point, centroid, dimension).
// Here the matrix cores compute the dot products x . mu~ in FP32
// (v_mfma_f32_16x16x4_f32; mu~ = the FP32 rounding of the FP64 centroid) and
// each pair gets the estimate s = (|x|^2 + |mu|^2) - 2 x . mu~ in FP32 with a
// rigorous bound E on its distance from the FP64 distance of the plain
// step (coefficients ea, eb from the host: FP32 rounding of the norms, of mu~,
// of the dot product's accumulation over dim terms and of s itself).  Every
// centroid whose lower bound s - E does not exceed the smallest upper bound
// s + E of the point is kept on a shortlist (the plain step's argmin is
// always on it); the point then takes its only candidate, or the plain
// step's FP64 argmin over its few candidates, or -- when more than MLIST
// centroids tie that closely (repeated centroids) -- over all centroids.
// The result is the plain step's assignment bit for bit.
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int MP = 64;     // points per block (16 per wavefront)
constexpr int MC = 64;     // centroids per pass (four 16-wide MFMA tiles)
constexpr int MK = 32;     // dimensions per LDS stage
constexpr int MLIST = 8;   // shortlist capacity per point

struct ShortArgs {
    const float *base;
    int64_t n;
    int dim;
    const double *mu;      // nh x dim FP64 centroids
    const float *mu32;     // their FP32 rounding
    const float *cn2;      // |mu|^2 per centroid (FP64 sum, rounded to FP32)
    const float *cn;       // |mu|
    const float *xn2;      // |x|^2 per point
    const float *xn;       // |x|
    int nh;
    float ea, eb;          // E = ea (|x|^2 + |mu|^2) + eb |x| |mu|
    int32_t *assign;
    int32_t *changed;
};

__global__ void point_norms_kernel(const float *base, int64_t n, int dim, float *xn2, float *xn)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double v = base[i * dim + j];
        s = s + v * v;
    }
    xn2[i] = (float)s;
    xn[i] = (float)sqrt(s);
}

__global__ void centroid_prep_kernel(const double *mu, int nh, int dim, float *mu32, float *cn2,
                                     float *cn)
{
#pragma clang fp contract(off)
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nh) return;
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double v = mu[(int64_t)c * dim + j];
        mu32[(int64_t)c * dim + j] = (float)v;
        s = s + v * v;
    }
    cn2[c] = (float)s;
    cn[c] = (float)sqrt(s);
}

__global__ void __launch_bounds__(256) assign_mfma_kernel(ShortArgs a)
{
#pragma clang fp contract(off)
    __shared__ float xs[MP][MK + 1];
    __shared__ float ms[MC][MK + 1];
    __shared__ float U[MP];
    __shared__ int cnt[MP];
    __shared__ int lc[MP][MLIST];
    __shared__ float ll[MP][MLIST];
    const float inf = __builtin_inff();
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int64_t p0 = (int64_t)blockIdx.x * MP;
    if (t < MP) {
        U[t] = inf;
        cnt[t] = 0;
    }
    // this lane's rows of the 16 x 16 output tiles: points 16w + 4 (lane >> 4) + i
    float X[4], XN[4];
    bool live[4];
    for (int i = 0; i < 4; ++i) {
        const int64_t pi = p0 + 16 * w + 4 * (lane >> 4) + i;
        live[i] = pi < a.n;
        X[i] = live[i] ? a.xn2[pi] : 0.f;
        XN[i] = live[i] ? a.xn[pi] : 0.f;
    }
    for (int c0 = 0; c0 < a.nh; c0 += MC) {
        v4f acc[4];
        for (int b = 0; b < 4; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < a.dim; k0 += MK) {
            __syncthreads();
            for (int e = t; e < MP * (MK / 4); e += 256) {
                const int r = e / (MK / 4), j = 4 * (e % (MK / 4));
                const int64_t gi = p0 + r;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (gi < a.n && k0 + j < a.dim)
                    v = *reinterpret_cast<const float4 *>(a.base + gi * a.dim + k0 + j);
                xs[r][j] = v.x;
                xs[r][j + 1] = v.y;
                xs[r][j + 2] = v.z;
                xs[r][j + 3] = v.w;
                const int c = c0 + r;
                float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
                if (c < a.nh && k0 + j < a.dim)
                    m = *reinterpret_cast<const float4 *>(a.mu32 + (int64_t)c * a.dim + k0 + j);
                ms[r][j] = m.x;
                ms[r][j + 1] = m.y;
                ms[r][j + 2] = m.z;
                ms[r][j + 3] = m.w;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < MK / 4; ++q) {
                const float av = xs[16 * w + (lane & 15)][4 * q + (lane >> 4)];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float bv = ms[16 * b + (lane & 15)][4 * q + (lane >> 4)];
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[b], 0, 0, 0);
                }
            }
        }
        // bounds of this pass's pairs; the smallest upper bound per point
        float lo[4][4], hmin[4];
        for (int i = 0; i < 4; ++i) {
            hmin[i] = inf;
            for (int b = 0; b < 4; ++b) {
                const int c = c0 + 16 * b + (lane & 15);
                lo[i][b] = inf;
                if (!live[i] || c >= a.nh) continue;
                const float C = a.cn2[c];
                const float s1 = X[i] + C;
                const float sv = s1 - 2.f * acc[b][i];
                const float e1 = a.ea * s1;
                const float e2 = a.eb * (XN[i] * a.cn[c]);
                const float E = e1 + e2;
                lo[i][b] = sv - E;
                const float hv = sv + E;
                hmin[i] = hv < hmin[i] ? hv : hmin[i];
            }
            for (int o = 1; o < 16; o <<= 1) {
                const float h2 = __shfl_xor(hmin[i], o);
                hmin[i] = h2 < hmin[i] ? h2 : hmin[i];
            }
        }
        __syncthreads();
        if ((lane & 15) == 0)
            for (int i = 0; i < 4; ++i) {
                const int P = 16 * w + 4 * (lane >> 4) + i;
                if (hmin[i] < U[P]) U[P] = hmin[i];
            }
        __syncthreads();
        // drop candidates whose lower bound now exceeds the point's bound
        if (t < MP && cnt[t] <= MLIST) {
            int m = 0;
            for (int r = 0; r < cnt[t]; ++r)
                if (ll[t][r] <= U[t]) {
                    lc[t][m] = lc[t][r];
                    ll[t][m] = ll[t][r];
                    ++m;
                }
            cnt[t] = m;
        }
        __syncthreads();
        for (int i = 0; i < 4; ++i) {
            const int P = 16 * w + 4 * (lane >> 4) + i;
            const float u = U[P];
            for (int b = 0; b < 4; ++b)
                if (lo[i][b] <= u && lo[i][b] < inf) {
                    const int slot = atomicAdd(&cnt[P], 1);
                    if (slot < MLIST) {
                        lc[P][slot] = c0 + 16 * b + (lane & 15);
                        ll[P][slot] = lo[i][b];
                    }
                }
        }
    }
    __syncthreads();
    if (t >= MP) return;
    const int64_t i = p0 + t;
    if (i >= a.n) return;
    const float *x = a.base + i * a.dim;
    int bc;
    if (cnt[t] == 1) {
        bc = lc[t][0];
    } else {
        // the plain step's FP64 argmin, over the shortlist or (when it
        // overflowed) over every centroid
        const bool all = cnt[t] > MLIST || cnt[t] == 0;
        const int m = all ? a.nh : cnt[t];
        double bv = __longlong_as_double(0x7ff0000000000000ll);
        bc = 0x7fffffff;
        for (int r = 0; r < m; ++r) {
            const int c = all ? r : lc[t][r];
            const double v = d2_to(x, a.mu + (int64_t)c * a.dim, a.dim);
            if (v < bv || (v == bv && c < bc)) {
                bv = v;
                bc = c;
            }
        }
    }
    if (a.assign[i] != bc) {
        a.assign[i] = bc;
        *a.changed = 1;
    }
}

__global__ void accumulate_kernel(const float *base, int64_t n, int dim, const int32_t *assign,
                                  double *sums, int64_t *count)
{
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (i >= n) return;
    const int lane = threadIdx.x & 63;
    const int c = assign[i];
    for (int j = lane; j < dim; j += 64)
        atomicAdd(&sums[(int64_t)c * dim + j], (double)base[i * dim + j]);
    if (lane == 0) atomicAdd((unsigned long long *)&count[c], 1ull);
}

__global__ void update_kernel(const double *sums, const int64_t *count, int nh, int dim, double *mu)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nh * dim) return;
    const int64_t c = e / dim;
    if (count[c] > 0) mu[e] = sums[e] / (double)count[c];
}

__global__ void hub_min_kernel(const float *base, int64_t n, int dim, const double *mu,
                               const int32_t *assign, unsigned long long *best_bits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = assign[i];
    double v = d2_to(base + i * dim, mu + (int64_t)c * dim, dim);
    atomicMin(&best_bits[c], (unsigned long long)__double_as_longlong(v));
}

__global__ void hub_id_kernel(const float *base, int64_t n, int dim, const double *mu,
                              const int32_t *assign, const unsigned long long *best_bits,
                              int32_t *hub)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = assign[i];
    double v = d2_to(base + i * dim, mu + (int64_t)c * dim, dim);
    if ((unsigned long long)__double_as_longlong(v) == best_bits[c]) atomicMin(&hub[c], (int32_t)i);
}

__global__ void init_mu_kernel(const float *base, int dim, const int32_t *init_ids, int nh,
                               double *mu)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nh * dim) return;
    const int64_t c = e / dim, j = e % dim;
    mu[e] = (double)base[(int64_t)init_ids[c] * dim + j];
}

__global__ void fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_f64(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// nearest point to mu_c that is not flagged in `taken`; (d2, id) order
struct Best {
    double v;
    int64_t id;
};

__global__ void __launch_bounds__(256) empty_scan_kernel(const float *base, int64_t n, int dim,
                                                         const double *m, const int32_t *taken,
                                                         Best *partial)
{
    __shared__ Best sh[256];
    Best b{__longlong_as_double(0x7ff0000000000000ll), 0x7fffffffffffffffll};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (taken[i]) continue;
        double v = d2_to(base + i * dim, m, dim);
        if (v < b.v || (v == b.v && i < b.id)) b = Best{v, i};
    }
    sh[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            Best o = sh[threadIdx.x + s];
            if (o.v < sh[threadIdx.x].v || (o.v == sh[threadIdx.x].v && o.id < sh[threadIdx.x].id))
                sh[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void mark_taken_kernel(const int32_t *hub, int nh, int32_t *taken)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nh && hub[c] >= 0) taken[hub[c]] = 1;
}

inline int grid_for(int64_t n, int per = 256, int cap = 8192)
{
    int64_t b = (n + per - 1) / per;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

// ---------------------------------------------------------------- HBKM
// distance of every point to the k children of its cluster (the same FP64
// arithmetic as the assignment above)
__global__ void child_dist_kernel(const float *base, int64_t n, int dim, const int32_t *parent,
                                  const double *mu, int k, double *D)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int j = (int)(e - i * k);
    D[e] = d2_to(base + i * dim, mu + ((int64_t)parent[i] * k + j) * dim, dim);
}

// Child j of cluster c starts at point init_ids[c * k + j], or at the
// parent's centroid when the parent has no member (init id -1).
__global__ void init_children_kernel(const float *base, int dim, const int32_t *init_ids, int64_t nc,
                                     int k, const double *parent_mu, double *mu)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc * dim) return;
    const int64_t c = e / dim, j = e % dim;
    const int32_t id = init_ids[c];
    mu[e] = id >= 0 ? (double)base[(int64_t)id * dim + j] : parent_mu[(c / k) * dim + j];
}

// One wavefront per parent cluster: its members (id order) join children in
// turn, each the child j of smallest d2(x, mu_j) + lambda * (2 (s_j - m/k) + 1)
// with s_j child j's size so far (ties to the smaller j).  Lane j keeps s_j;
// the distances of 64 members at a time are staged in LDS, so the sequential
// chain only waits on LDS and shuffles.
constexpr int HB_CHUNK = 64;

__global__ void __launch_bounds__(64) balanced_pass_kernel(const int32_t *members,
                                                           const int64_t *start, int64_t np,
                                                           const double *D, int k, double lambda,
                                                           int32_t *child)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char hb_lds[];
    double *ds = reinterpret_cast<double *>(hb_lds);                  // HB_CHUNK x k
    int32_t *ms = reinterpret_cast<int32_t *>(ds + HB_CHUNK * k);     // HB_CHUNK
    const int64_t p = blockIdx.x;
    if (p >= np) return;
    const int lane = threadIdx.x;
    const int64_t s0 = start[p];
    const int64_t m = start[p + 1] - s0;
    const double target = (double)m / (double)k;
    const double inf = __longlong_as_double(0x7ff0000000000000ll);
    int64_t s = 0;
    for (int64_t r0 = 0; r0 < m; r0 += HB_CHUNK) {
        const int cnt = (int)(m - r0 < HB_CHUNK ? m - r0 : HB_CHUNK);
        if (lane < cnt) ms[lane] = members[s0 + r0 + lane];
        __syncthreads();
        for (int e = lane; e < cnt * k; e += 64) {
            const int q = e / k, j = e - q * k;
            ds[e] = D[(int64_t)ms[q] * k + j];
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            double v = inf;
            int idx = lane;
            if (lane < k) {
                const double dev = (double)s - target;
                const double pen = lambda * (2.0 * dev + 1.0);
                v = ds[q * k + lane] + pen;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(v, o);
                const int oi = __shfl_xor(idx, o);
                if (ov < v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (lane == idx) ++s;
            if (lane == 0) child[ms[q]] = (int32_t)(p * k + idx);
        }
        __syncthreads();
    }
}

}  // namespace

namespace {

// Definition 3 hubs of given clusters: the member nearest the cluster's
// mean by (d2, id); an empty cluster takes the nearest point that is not yet
// a hub (clusters in index order).
ann_status hubs_of_clusters(const float *base, int64_t n, int dim, int nh, const double *mu,
                            const int32_t *assign, int32_t *hub_ids, unsigned long long *bits,
                            int32_t *taken, Best *partial, hipStream_t st)
{
    hipLaunchKernelGGL(fill_u64, dim3(grid_for(nh)), dim3(256), 0, st, bits, (int64_t)nh,
                       0xFFFFFFFFFFFFFFFFull);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(fill_i32, dim3(grid_for(nh)), dim3(256), 0, st, hub_ids, (int64_t)nh,
                       0x7fffffff);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(hub_min_kernel, dim3(grid_for(n, 256, 1 << 22)), dim3(256), 0, st, base, n, dim,
                       mu, assign, bits);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(hub_id_kernel, dim3(grid_for(n, 256, 1 << 22)), dim3(256), 0, st, base, n, dim,
                       mu, assign, bits, hub_ids);
    ANN_LAUNCHED();
    // empty clusters (no member): nearest point that is not yet a hub
    std::vector<int32_t> hh((size_t)nh);
    ANN_HIP(hipMemcpyAsync(hh.data(), hub_ids, sizeof(int32_t) * nh, hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    bool any_empty = false;
    for (int c = 0; c < nh; ++c) any_empty |= (hh[c] == 0x7fffffff);
    if (any_empty) {
        hipLaunchKernelGGL(fill_i32, dim3(grid_for(n)), dim3(256), 0, st, taken, n, 0);
        ANN_LAUNCHED();
        // flag the hubs of non-empty clusters
        for (int c = 0; c < nh; ++c)
            if (hh[c] == 0x7fffffff) hh[c] = -1;
        ANN_HIP(hipMemcpyAsync(hub_ids, hh.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(mark_taken_kernel, dim3(grid_for(nh)), dim3(256), 0, st, hub_ids, nh, taken);
        ANN_LAUNCHED();
        const int blocks = grid_for(n, 256, 1024);
        for (int c = 0; c < nh; ++c) {
            if (hh[c] >= 0) continue;
            hipLaunchKernelGGL(empty_scan_kernel, dim3(blocks), dim3(256), 0, st, base, n, dim,
                               mu + (int64_t)c * dim, taken, partial);
            ANN_LAUNCHED();
            std::vector<Best> pb((size_t)blocks);
            ANN_HIP(hipMemcpyAsync(pb.data(), partial, sizeof(Best) * blocks, hipMemcpyDeviceToHost, st));
            ANN_HIP(hipStreamSynchronize(st));
            Best b = pb[0];
            for (int q = 1; q < blocks; ++q)
                if (pb[q].v < b.v || (pb[q].v == b.v && pb[q].id < b.id)) b = pb[q];
            hh[c] = (int32_t)b.id;
            int32_t one = 1;
            ANN_HIP(hipMemcpyAsync(taken + b.id, &one, 4, hipMemcpyHostToDevice, st));
            ANN_HIP(hipStreamSynchronize(st));
        }
        ANN_HIP(hipMemcpyAsync(hub_ids, hh.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice, st));
        ANN_HIP(hipStreamSynchronize(st));
    }
    return ANN_OK;
}

}  // namespace

size_t select_hubs_ws(int64_t n, int dim, int nh)
{
    size_t b = round_up((size_t)nh * dim * 8, 256) * 2;       // mu, sums
    b += round_up((size_t)nh * 8, 256) * 2;                   // count, best bits
    b += round_up((size_t)n * 4, 256) * 2;                    // assign, taken
    b += round_up(4096 * sizeof(Best), 256) + 1024;
    b += round_up((size_t)nh * dim * 4, 256);                 // FP32 centroids
    b += round_up((size_t)nh * 4, 256) * 2;                   // their norms
    b += round_up((size_t)n * 4, 256) * 2;                    // point norms
    return b;
}

ann_status select_hubs_run(const float *base, int64_t n, int dim, int nh, int iters,
                           const int32_t *init_ids, int32_t *hub_ids, double *centroids_out,
                           int32_t *assign_out, int32_t *steps_out, void *ws, hipStream_t st)
{
    Carve cv{static_cast<unsigned char *>(ws)};
    double *mu = centroids_out ? centroids_out : cv.take<double>((size_t)nh * dim);
    if (centroids_out) cv.take<double>((size_t)nh * dim);
    double *sums = cv.take<double>((size_t)nh * dim);
    int64_t *count = cv.take<int64_t>((size_t)nh);
    unsigned long long *bits = cv.take<unsigned long long>((size_t)nh);
    int32_t *assign = assign_out ? assign_out : cv.take<int32_t>((size_t)n);
    if (assign_out) cv.take<int32_t>((size_t)n);
    int32_t *taken = cv.take<int32_t>((size_t)n);
    Best *partial = cv.take<Best>(4096);
    int32_t *changed = cv.take<int32_t>(64);
    float *mu32 = cv.take<float>((size_t)nh * dim);
    float *cn2 = cv.take<float>((size_t)nh);
    float *cn = cv.take<float>((size_t)nh);
    float *xn2 = cv.take<float>((size_t)n);
    float *xn = cv.take<float>((size_t)n);
    // the matrix-core assignment needs whole float4 rows
    const bool mfma = dim % 4 == 0 && aligned(base, 16);
    ShortArgs sa{};
    if (mfma) {
        hipLaunchKernelGGL(point_norms_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           base, n, dim, xn2, xn);
        ANN_LAUNCHED();
        // bound coefficients (unit roundoff u = 2^-24): the norms and mu~ are
        // FP32 roundings, the dot product accumulates dim FP32 terms (gamma),
        // s and the bounds themselves add a few roundings; margins of >= 30 %
        const double u = std::ldexp(1.0, -24);
        const double K = (double)dim + 2.0;
        const double gam = K * u / (1.0 - K * u);
        const double gp = gam * (1.0 + u) + u;
        sa = ShortArgs{base, n, dim, nullptr, mu32, cn2, cn, xn2, xn, nh,
                       (float)(8.0 * u), (float)(2.1 * gp + 12.0 * u), nullptr, changed};
    }

    const int64_t md = (int64_t)nh * dim;
    hipLaunchKernelGGL(init_mu_kernel, dim3(grid_for(md, 256, 1 << 20)), dim3(256), 0, st, base, dim,
                       init_ids, nh, mu);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(fill_i32, dim3(grid_for(n)), dim3(256), 0, st, assign, n, -1);
    ANN_LAUNCHED();
    int steps = 0;
    for (int t = 0; t < iters; ++t) {
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, changed, 1, 0);
        ANN_LAUNCHED();
        if (mfma) {
            hipLaunchKernelGGL(centroid_prep_kernel, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0,
                               st, mu, nh, dim, mu32, cn2, cn);
            ANN_LAUNCHED();
            sa.mu = mu;
            sa.assign = assign;
            hipLaunchKernelGGL(assign_mfma_kernel, dim3((unsigned)((n + MP - 1) / MP)), dim3(256), 0,
                               st, sa);
        } else {
            hipLaunchKernelGGL(assign_kernel, dim3((unsigned)((n + KP - 1) / KP)), dim3(256), 0, st,
                               base, n, dim, mu, nh, assign, changed);
        }
        ANN_LAUNCHED();
        ++steps;
        hipLaunchKernelGGL(fill_f64, dim3(grid_for(md)), dim3(256), 0, st, sums, md);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(fill_u64, dim3(grid_for(nh)), dim3(256), 0, st,
                           (unsigned long long *)count, (int64_t)nh, 0ull);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(accumulate_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base, n,
                           dim, assign, sums, count);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(update_kernel, dim3(grid_for(md, 256, 1 << 20)), dim3(256), 0, st, sums,
                           count, nh, dim, mu);
        ANN_LAUNCHED();
        int32_t h = 0;
        ANN_HIP(hipMemcpyAsync(&h, changed, 4, hipMemcpyDeviceToHost, st));
        ANN_HIP(hipStreamSynchronize(st));
        if (!h) break;
    }
    ann_status hs = hubs_of_clusters(base, n, dim, nh, mu, assign, hub_ids, bits, taken, partial, st);
    if (hs != ANN_OK) return hs;
    if (steps_out) *steps_out = steps;
    return ANN_OK;
}

}  // namespace ann

using namespace ann;

namespace ann {
namespace {

int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

size_t hbkm_ws(int64_t n, int dim, int k, int levels)
{
    const int64_t nc = ipow(k, levels), np = ipow(k, levels - 1);
    size_t b = round_up((size_t)n * k * 8, 256);                 // distances to the children
    b += round_up((size_t)n * 4, 256) * 4;                        // parent, child, members, taken
    b += round_up((size_t)(np + 1) * 8, 256);                     // member offsets
    b += round_up((size_t)nc * 4, 256);                           // initial members
    b += round_up((size_t)nc * dim * 8, 256) * 3;                 // mu, parent mu, sums
    b += round_up((size_t)nc * 8, 256) * 2;                       // count, best bits
    b += round_up(4096 * sizeof(Best), 256);
    return b + 1024;
}

ann_status hbkm_run(const float *base, int64_t n, int dim, int k, int levels, double lambda,
                    int iters, int32_t *hub_ids, double *centroids_out, int32_t *assign_out,
                    void *ws, hipStream_t st)
{
    const int64_t nc_max = ipow(k, levels), np_max = ipow(k, levels - 1);
    Carve cv{static_cast<unsigned char *>(ws)};
    double *D = cv.take<double>((size_t)n * k);
    int32_t *cur = cv.take<int32_t>((size_t)n);
    int32_t *nxt = cv.take<int32_t>((size_t)n);
    int32_t *mem_d = cv.take<int32_t>((size_t)n);
    int32_t *taken = cv.take<int32_t>((size_t)n);
    int64_t *start_d = cv.take<int64_t>((size_t)np_max + 1);
    int32_t *init_d = cv.take<int32_t>((size_t)nc_max);
    double *mu = cv.take<double>((size_t)nc_max * dim);
    double *pmu = cv.take<double>((size_t)nc_max * dim);
    double *sums = cv.take<double>((size_t)nc_max * dim);
    int64_t *count = cv.take<int64_t>((size_t)nc_max);
    unsigned long long *bits = cv.take<unsigned long long>((size_t)nc_max);
    Best *partial = cv.take<Best>(4096);

    hipLaunchKernelGGL(fill_i32, dim3(grid_for(n)), dim3(256), 0, st, cur, n, 0);
    ANN_LAUNCHED();
    std::vector<int32_t> lab((size_t)n), members((size_t)n), init;
    std::vector<int64_t> start;
    const size_t pass_lds = (size_t)HB_CHUNK * k * 8 + HB_CHUNK * 4;
    int64_t np = 1;
    for (int l = 1; l <= levels; ++l) {
        const int64_t nc = np * k;
        // members of every parent in id order, and each child's first member
        ANN_HIP(hipMemcpyAsync(lab.data(), cur, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
        ANN_HIP(hipStreamSynchronize(st));
        start.assign((size_t)np + 1, 0);
        for (int64_t i = 0; i < n; ++i) start[(size_t)lab[(size_t)i] + 1]++;
        for (int64_t p = 0; p < np; ++p) start[(size_t)p + 1] += start[(size_t)p];
        {
            std::vector<int64_t> fill(start.begin(), start.end() - 1);
            for (int64_t i = 0; i < n; ++i) members[(size_t)fill[(size_t)lab[(size_t)i]]++] = (int32_t)i;
        }
        init.assign((size_t)nc, -1);
        for (int64_t p = 0; p < np; ++p) {
            const int64_t m = start[(size_t)p + 1] - start[(size_t)p];
            if (m == 0) continue;
            for (int j = 0; j < k; ++j)
                init[(size_t)(p * k + j)] = members[(size_t)(start[(size_t)p] + (2 * j + 1) * m / (2 * k))];
        }
        ANN_HIP(hipMemcpyAsync(mem_d, members.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
        ANN_HIP(hipMemcpyAsync(start_d, start.data(), sizeof(int64_t) * (size_t)(np + 1),
                               hipMemcpyHostToDevice, st));
        ANN_HIP(hipMemcpyAsync(init_d, init.data(), sizeof(int32_t) * (size_t)nc, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(init_children_kernel, dim3((unsigned)((nc * dim + 255) / 256)), dim3(256), 0,
                           st, base, dim, init_d, nc, k, pmu, mu);
        ANN_LAUNCHED();
        const int64_t md = nc * dim;
        for (int t = 0; t < iters; ++t) {
            hipLaunchKernelGGL(child_dist_kernel, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, st,
                               base, n, dim, cur, mu, k, D);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(balanced_pass_kernel, dim3((unsigned)np), dim3(64), pass_lds, st, mem_d,
                               start_d, np, D, k, lambda, nxt);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(fill_f64, dim3(grid_for(md)), dim3(256), 0, st, sums, md);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(fill_u64, dim3(grid_for(nc)), dim3(256), 0, st,
                               (unsigned long long *)count, nc, 0ull);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(accumulate_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base,
                               n, dim, nxt, sums, count);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(update_kernel, dim3((unsigned)((md + 255) / 256)), dim3(256), 0, st, sums,
                               count, (int)nc, dim, mu);
            ANN_LAUNCHED();
        }
        std::swap(cur, nxt);
        std::swap(mu, pmu);
        np = nc;
    }
    // cur: final clusters, pmu: their centroids
    ANN_HIP(hipMemcpyAsync(assign_out, cur, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
    if (centroids_out)
        ANN_HIP(hipMemcpyAsync(centroids_out, pmu, sizeof(double) * (size_t)np * dim,
                               hipMemcpyDeviceToDevice, st));
    ann_status hs = hubs_of_clusters(base, n, dim, (int)np, pmu, cur, hub_ids, bits, taken, partial, st);
    if (hs != ANN_OK) return hs;
    ANN_HIP(hipStreamSynchronize(st));
    return ANN_OK;
}

bool hbkm_shape_ok(int64_t n, int32_t k, int32_t levels)
{
    if (k < 2 || k > 64 || levels < 1 || levels > 20) return false;
    int64_t nc = 1;
    for (int l = 0; l < levels; ++l) {
        nc *= k;
        if (nc > n || nc > (1 << 20)) return false;
    }
    return true;
}

}  // namespace
}  // namespace ann

extern "C" size_t ann_select_hubs_hbkm_workspace_size(int64_t n, int32_t dim, int32_t k,
                                                      int32_t levels)
{
    if (n < 1 || dim < 1 || !hbkm_shape_ok(n, k, levels)) return 0;
    return hbkm_ws(n, dim, k, levels);
}

extern "C" ann_status ann_select_hubs_hbkm(const float *base, int64_t n, int32_t dim, int32_t k,
                                           int32_t levels, double lambda, int32_t iters,
                                           int32_t *hub_ids, double *centroids, int32_t *assign,
                                           void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && hub_ids && assign && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(hbkm_shape_ok(n, k, levels),
                "need 2 <= k <= 64, levels >= 1 and k^levels <= min(n, 2^20)");
    ANN_REQUIRE(lambda >= 0.0 && lambda < 1e300, "lambda must be finite and >= 0");
    ANN_REQUIRE(iters >= 1, "iters must be >= 1");
    ANN_REQUIRE(ws_bytes >= hbkm_ws(n, dim, k, levels), "workspace too small");
    return hbkm_run(base, n, dim, k, levels, lambda, iters, hub_ids, centroids, assign, workspace,
                    static_cast<hipStream_t>(stream));
}

extern "C" ann_status ann_select_hubs(const float *base, int64_t n, int32_t dim, int32_t n_hubs,
                                      int32_t iters, const int32_t *init_ids, int32_t *hub_ids,
                                      double *centroids, int32_t *assign, int32_t *steps,
                                      void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && init_ids && hub_ids && workspace, "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(n_hubs >= 1 && n_hubs <= n, "n_hubs must be in [1, n]");
    ANN_REQUIRE(iters >= 1, "iters must be >= 1");
    ANN_REQUIRE(ws_bytes >= ann_workspace_size(ANN_OP_SELECT_HUBS, n, dim, n_hubs, 0),
                "workspace too small");
    return select_hubs_run(base, n, dim, n_hubs, iters, init_ids, hub_ids, centroids, assign, steps,
                           workspace, static_cast<hipStream_t>(stream));
}

// Seeded k-means start.  The generator is SplitMix64 (Steele, Lea and Flood,
// OOPSLA 2014): the state advances by the golden-ratio increment and each
// output is the state through the generator's finaliser.  The i-th output x
// picks t in [0, j] as the high word of x * (j + 1) (Lemire's multiply-shift,
// 2019, no rejection), and Floyd's sampling (Bentley and Floyd, CACM 1987)
// takes t, or j when t is already taken, for j = n - n_hubs .. n - 1.
extern "C" ann_status ann_hub_init_ids(int64_t n, int32_t n_hubs, uint64_t seed, int32_t *ids)
{
    ANN_REQUIRE(ids != nullptr, "ids is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(n_hubs >= 1 && n_hubs <= n, "n_hubs must be in [1, n]");
    std::unordered_set<int64_t> taken;
    taken.reserve((size_t)n_hubs * 2);
    uint64_t state = seed;
    int32_t i = 0;
    for (int64_t j = n - n_hubs; j < n; ++j) {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const int64_t t = (int64_t)(((unsigned __int128)z * (uint64_t)(j + 1)) >> 64);
        const int64_t v = taken.count(t) ? j : t;
        taken.insert(v);
        ids[i++] = (int32_t)v;
    }
    return ANN_OK;
}
