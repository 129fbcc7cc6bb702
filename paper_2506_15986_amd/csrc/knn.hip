// Exact brute-force k nearest neighbours on the GPU (ground truth for
// recall, Eq. 1, and the candidate lists of the proximity graph).
//
// Two distance engines feed the shared top-K selection of knn_core.h:
//   * integer engine: every value is an integer in [0, 255]; vectors are
//     shifted by -128 into int8 and the dot products run on the int8 matrix
//     cores (v_mfma_i32_16x16x32_i8); d2 = |x'|^2 + |y'|^2 - 2 x'.y' is exact
//     in int32;
//   * FP64 engine: any data; d2 = sum_j (x_j - y_j)^2 in FP64.  On data held
//     on a dyadic grid (values m * 2^-G with 2G + log2(d (2B)^2) <= 53) every
//     partial sum is exact, so the result equals the FP64 sum in any order.
// Both give the exact top K by (d2, id).
#include "common.h"
#include "knn.h"
#include "knn_core.h"

namespace ann {
namespace {

using knn::Ent;

// ---------------------------------------------------------------- helpers
__global__ void check_uint8_kernel(const float *x, int64_t count, int *bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int local = 0;
    for (; i < count; i += stride) {
        float v = x[i];
        if (!(v >= 0.f && v <= 255.f && v == rintf(v))) local = 1;
    }
    if (local) atomicOr(bad, 1);
}

// int8 copy (x - 128) and squared norms of the shifted rows
__global__ void to_int8_kernel(const float *x, int64_t rows, int dim, int8_t *out, int32_t *norm)
{
    int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x / 64);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    int acc = 0;
    for (int j = lane; j < dim; j += 64) {
        int v = (int)x[r * dim + j] - 128;
        out[r * dim + j] = (int8_t)v;
        acc += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) norm[r] = acc;
}

struct RowState {
    Ent thr[knn::kRows];
    int cnt[knn::kRows];
};

// append (key, col) to row `lr` (local row) if it beats the threshold
__device__ inline void offer(RowState &rs, Ent *buf, int64_t grow, int lr, int cap, uint64_t key,
                             uint32_t col)
{
    Ent e;
    e.k = key;
    e.id = col;
    e.pad = 0;
    if (knn::less(e, rs.thr[lr])) {
        int slot = atomicAdd(&rs.cnt[lr], 1);
        buf[grow * cap + slot] = e;
    }
}

// wave w: merge its rows whose buffers cannot take another tile
__device__ inline void merge_full_rows(RowState &rs, Ent *buf, int64_t row0, int64_t rows, int cap,
                                       int K, int tile, Ent *scratch, bool final_pass)
{
    const int w = threadIdx.x >> 6;
    for (int r = w * knn::kRowsPerWave; r < (w + 1) * knn::kRowsPerWave; ++r) {
        int64_t g = row0 + r;
        if (g >= rows) break;
        if (final_pass || rs.cnt[r] > cap - tile) {
            int c = rs.cnt[r];
            Ent thr = rs.thr[r];
            knn::merge_row(buf + g * cap, cap, K, scratch, thr, c);
            if (__lane_id() == 0) {
                rs.thr[r] = thr;
                rs.cnt[r] = c;
            }
            knn::wsync();
        }
    }
}

__device__ inline void write_rows(const RowState &rs, const Ent *buf, int64_t row0, int64_t rows,
                                  int cap, int K, bool int_keys, int32_t *out_ids, float *out_f,
                                  double *out_d)
{
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    for (int r = w * knn::kRowsPerWave; r < (w + 1) * knn::kRowsPerWave; ++r) {
        int64_t g = row0 + r;
        if (g >= rows) break;
        int c = rs.cnt[r];
        for (int t = lane; t < K; t += 64) {
            int32_t id = -1;
            double v = __longlong_as_double(0x7ff0000000000000ll);
            if (t < c) {
                Ent e = buf[g * cap + t];
                id = (int32_t)e.id;
                v = int_keys ? (double)e.k : knn::value_of(e.k);
            }
            out_ids[g * K + t] = id;
            if (out_f) out_f[g * K + t] = (float)v;
            if (out_d) out_d[g * K + t] = v;
        }
    }
}

// base column that query row g must skip (-1: none)
__device__ inline int64_t self_column(const KnnArgs &a, int64_t g)
{
    if (!a.exclude_self || g >= a.rows) return -1;
    return a.self_col ? (int64_t)a.self_col[g] : g;
}

// ---------------------------------------------------------------- FP64 engine
constexpr int F_BN = 64;    // columns per tile
constexpr int F_DK = 32;    // dims per LDS stage

__global__ void __launch_bounds__(256) knn_f64_kernel(KnnArgs a)
{
    __shared__ float As[knn::kRows][F_DK + 1];
    __shared__ float Bs[F_BN][F_DK + 1];
    __shared__ RowState rs;
    extern __shared__ __align__(16) unsigned char dyn[];
    Ent *scratch = reinterpret_cast<Ent *>(dyn) + (threadIdx.x >> 6) * a.cap;

    const int t = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * knn::kRows;
    const int r0 = (t / 16) * 4;     // 4 rows per thread (rows of wave t/64)
    const int c0 = (t % 16) * 4;     // 4 columns per thread
    if (t < knn::kRows) {
        rs.thr[t] = knn::ent_max();
        rs.cnt[t] = 0;
    }
    int64_t selfc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) selfc[i] = self_column(a, row0 + r0 + i);
    __syncthreads();
    for (int64_t col0 = 0; col0 < a.n; col0 += F_BN) {
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int dk = 0; dk < a.dim; dk += F_DK) {
            for (int e = t; e < knn::kRows * F_DK; e += 256) {
                int r = e / F_DK, j = e % F_DK;
                int64_t g = row0 + r;
                As[r][j] = (g < a.rows && dk + j < a.dim) ? a.queries[g * a.dim + dk + j] : 0.f;
            }
            for (int e = t; e < F_BN * F_DK; e += 256) {
                int c = e / F_DK, j = e % F_DK;
                int64_t g = col0 + c;
                Bs[c][j] = (g < a.n && dk + j < a.dim) ? a.base[g * a.dim + dk + j] : 0.f;
            }
            __syncthreads();
#pragma unroll 4
            for (int j = 0; j < F_DK; ++j) {
                double av[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = (double)As[r0 + i][j];
#pragma unroll
                for (int i = 0; i < 4; ++i) bv[i] = (double)Bs[c0 + i][j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        double d = av[i] - bv[k];
                        acc[i][k] += d * d;
                    }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int64_t g = row0 + r0 + i;
            if (g >= a.rows) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int64_t col = col0 + c0 + k;
                if (col >= a.n || col == selfc[i]) continue;
                offer(rs, a.buf, g, r0 + i, a.cap, knn::key_of(acc[i][k]), (uint32_t)col);
            }
        }
        knn::wsync();
        merge_full_rows(rs, a.buf, row0, a.rows, a.cap, a.K, F_BN, scratch, false);
    }
    merge_full_rows(rs, a.buf, row0, a.rows, a.cap, a.K, F_BN, scratch, true);
    write_rows(rs, a.buf, row0, a.rows, a.cap, a.K, false, a.out_ids, a.out_f, a.out_d);
}

// ---------------------------------------------------------------- int8 MFMA engine
// Tile: 64 rows x 128 columns, k-steps of 32 bytes.  Wave w computes rows
// [16w, 16w+16) against all 128 columns as 8 output blocks of 16x16.
// v_mfma_i32_16x16x32_i8 operands: lane l supplies 8 bytes of row (l % 16)
// of A (resp. column (l % 16) of B) at k offset 8 * (l / 16); the int32
// result element i of lane l is C[4 * (l / 16) + i][l % 16].
constexpr int I_BN = 128;
constexpr int I_MAXD = 256;

typedef int v4i __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) knn_i8_kernel(KnnArgs a)
{
    __shared__ __align__(16) int8_t Bs[I_BN][I_MAXD + 16];
    __shared__ int32_t Bn[I_BN];
    __shared__ RowState rs;
    extern __shared__ __align__(16) unsigned char dyn[];
    Ent *scratch = reinterpret_cast<Ent *>(dyn) + (threadIdx.x >> 6) * a.cap;

    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = t & 63;
    const int64_t row0 = (int64_t)blockIdx.x * knn::kRows;
    const int ksteps = a.dim / 32;
    if (t < knn::kRows) {
        rs.thr[t] = knn::ent_max();
        rs.cnt[t] = 0;
    }
    // A operand for all k-steps: row (16w + l%16), bytes 8*(l/16) + 32*s
    long long areg[I_MAXD / 32];
    const int64_t arow = row0 + 16 * w + (lane & 15);
    for (int s = 0; s < I_MAXD / 32; ++s) {
        long long v = 0;
        if (s < ksteps && arow < a.rows)
            v = *reinterpret_cast<const long long *>(a.q8 + arow * a.dim + 32 * s + 8 * (lane >> 4));
        areg[s] = v;
    }
    int32_t anorm[4];
    int64_t selfc[4];
    for (int i = 0; i < 4; ++i) {
        int64_t g = row0 + 16 * w + 4 * (lane >> 4) + i;
        anorm[i] = g < a.rows ? a.qnorm[g] : 0;
        selfc[i] = self_column(a, g);
    }
    __syncthreads();
    const int chunks16 = a.dim / 16;
    for (int64_t col0 = 0; col0 < a.n; col0 += I_BN) {
        for (int e = t; e < I_BN * chunks16; e += 256) {
            int c = e / chunks16, j = e % chunks16;
            int64_t g = col0 + c;
            v4i v = {0, 0, 0, 0};
            if (g < a.n) v = *reinterpret_cast<const v4i *>(a.b8 + g * a.dim + 16 * j);
            *reinterpret_cast<v4i *>(&Bs[c][16 * j]) = v;
        }
        for (int c = t; c < I_BN; c += 256) {
            int64_t g = col0 + c;
            Bn[c] = g < a.n ? a.bnorm[g] : 0;
        }
        __syncthreads();
#pragma unroll 2
        for (int blk = 0; blk < I_BN / 16; ++blk) {
            v4i acc = {0, 0, 0, 0};
            const int bc = 16 * blk + (lane & 15);
            for (int s = 0; s < ksteps; ++s) {
                long long bv = *reinterpret_cast<const long long *>(&Bs[bc][32 * s + 8 * (lane >> 4)]);
                acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(areg[s], bv, acc, 0, 0, 0);
            }
            const int64_t col = col0 + bc;
            if (col < a.n) {
                const int32_t bn = Bn[bc];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int lr = 16 * w + 4 * (lane >> 4) + i;
                    int64_t g = row0 + lr;
                    if (g >= a.rows || col == selfc[i]) continue;
                    int32_t d2 = anorm[i] + bn - 2 * acc[i];
                    offer(rs, a.buf, g, lr, a.cap, (uint64_t)(uint32_t)d2, (uint32_t)col);
                }
            }
        }
        knn::wsync();
        merge_full_rows(rs, a.buf, row0, a.rows, a.cap, a.K, I_BN, scratch, false);
        __syncthreads();
    }
    merge_full_rows(rs, a.buf, row0, a.rows, a.cap, a.K, I_BN, scratch, true);
    write_rows(rs, a.buf, row0, a.rows, a.cap, a.K, true, a.out_ids, a.out_f, a.out_d);
}

}  // namespace

size_t knn_cap(int K, bool int_engine)
{
    int tile = int_engine ? I_BN : F_BN;
    size_t c = 2;
    while (c < (size_t)(K + tile)) c <<= 1;
    return c;
}

size_t knn_workspace(int64_t n, int64_t rows, int dim, int K)
{
    size_t cap = knn_cap(K, true) > knn_cap(K, false) ? knn_cap(K, true) : knn_cap(K, false);
    size_t b = round_up((size_t)rows * cap * sizeof(Ent), 256);
    b += round_up((size_t)n * dim, 256) + round_up((size_t)n * 4, 256);        // base int8 + norms
    b += round_up((size_t)rows * dim, 256) + round_up((size_t)rows * 4, 256);  // query int8 + norms
    b += 256;
    return b;
}

ann_status data_is_uint8(const float *x, int64_t count, int *flag_dev, bool *result, hipStream_t st)
{
    ANN_HIP(hipMemsetAsync(flag_dev, 0, sizeof(int), st));
    int blocks = (int)((count + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(check_uint8_kernel, dim3(blocks), dim3(256), 0, st, x, count, flag_dev);
    ANN_LAUNCHED();
    int h = 0;
    ANN_HIP(hipMemcpyAsync(&h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    *result = (h == 0);
    return ANN_OK;
}

// Exact kNN of `rows` query rows against base; ids and distances written
// to out_ids and out_f (float) and/or out_d (double).  Synchronises.
ann_status knn_run(const float *base, int64_t n, int dim, const float *queries, int64_t rows,
                   int K, bool exclude_self, int32_t *out_ids, float *out_f, double *out_d,
                   void *ws, size_t ws_bytes, hipStream_t st, int force_engine,
                   const int32_t *self_col)
{
    ANN_REQUIRE(ws_bytes >= knn_workspace(n, rows, dim, K), "kNN workspace too small");
    unsigned char *p = static_cast<unsigned char *>(ws);
    size_t cap_i = knn_cap(K, true), cap_f = knn_cap(K, false);
    size_t cap = cap_i > cap_f ? cap_i : cap_f;
    Ent *buf = reinterpret_cast<Ent *>(p);
    p += round_up((size_t)rows * cap * sizeof(Ent), 256);
    int8_t *b8 = reinterpret_cast<int8_t *>(p);
    p += round_up((size_t)n * dim, 256);
    int32_t *bn = reinterpret_cast<int32_t *>(p);
    p += round_up((size_t)n * 4, 256);
    int8_t *q8 = reinterpret_cast<int8_t *>(p);
    p += round_up((size_t)rows * dim, 256);
    int32_t *qn = reinterpret_cast<int32_t *>(p);
    p += round_up((size_t)rows * 4, 256);
    int *flag = reinterpret_cast<int *>(p);

    bool use_int = false;
    if (force_engine != 2 && dim % 32 == 0 && dim <= I_MAXD) {
        bool bu = false, qu = false;
        ann_status s = data_is_uint8(base, n * dim, flag, &bu, st);
        if (s != ANN_OK) return s;
        if (bu) {
            s = data_is_uint8(queries, rows * dim, flag, &qu, st);
            if (s != ANN_OK) return s;
        }
        use_int = bu && qu;
    }
    if (force_engine == 1 && !use_int) return fail(ANN_EINVAL, "int8 engine needs integer data in [0,255]");
    KnnArgs a{};
    a.base = base;
    a.n = n;
    a.dim = dim;
    a.queries = queries;
    a.rows = rows;
    a.K = K;
    a.exclude_self = exclude_self ? 1 : 0;
    a.self_col = self_col;
    a.buf = buf;
    a.out_ids = out_ids;
    a.out_f = out_f;
    a.out_d = out_d;
    const int blocks = (int)((rows + knn::kRows - 1) / knn::kRows);
    if (use_int) {
        a.cap = (int)cap_i;
        hipLaunchKernelGGL(to_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base, n, dim,
                           b8, bn);
        ANN_LAUNCHED();
        hipLaunchKernelGGL(to_int8_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, queries,
                           rows, dim, q8, qn);
        ANN_LAUNCHED();
        a.b8 = b8;
        a.bnorm = bn;
        a.q8 = q8;
        a.qnorm = qn;
        size_t lds = 4 * (size_t)a.cap * sizeof(Ent);
        ANN_HIP(hipFuncSetAttribute((const void *)knn_i8_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(knn_i8_kernel, dim3(blocks), dim3(256), lds, st, a);
        ANN_LAUNCHED();
    } else {
        a.cap = (int)cap_f;
        size_t lds = 4 * (size_t)a.cap * sizeof(Ent);
        ANN_HIP(hipFuncSetAttribute((const void *)knn_f64_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(knn_f64_kernel, dim3(blocks), dim3(256), lds, st, a);
        ANN_LAUNCHED();
    }
    ANN_HIP(hipStreamSynchronize(st));
    return ANN_OK;
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_gt_knn(const float *base, int64_t n, int32_t dim, const float *queries,
                                 int32_t nq, int32_t k, int32_t exclude_self, int32_t *out_ids,
                                 float *out_dist, void *workspace, size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(base && workspace, "a required pointer is NULL");
    ANN_REQUIRE(nq == 0 || (queries && out_ids && out_dist), "a required pointer is NULL");
    ANN_REQUIRE(n >= 1 && n <= 0x7FFFFFFF, "n must be in [1, 2^31)");
    ANN_REQUIRE(dim >= 1, "dim must be >= 1");
    ANN_REQUIRE(k >= 1 && k <= 1024, "k must be in [1, 1024]");
    ANN_REQUIRE(nq >= 0, "nq must be >= 0");
    ANN_REQUIRE(!exclude_self || nq <= n, "exclude_self needs nq <= n");
    ANN_REQUIRE(ws_bytes >= ann_workspace_size(ANN_OP_GT_KNN, n, dim, nq, k), "workspace too small");
    if (nq == 0) return ANN_OK;
    return knn_run(base, n, dim, queries, nq, k, exclude_self != 0, out_ids, out_dist, nullptr,
                   workspace, ws_bytes, static_cast<hipStream_t>(stream), 0);
}
