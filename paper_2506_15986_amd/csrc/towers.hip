// Two-tower entry model (two-tower score of the preliminaries; projection
// network of the high-tier graph section): forward, backward, contrastive
// loss and Adam, all deterministic (no floating-point atomics; every
// reduction runs in a fixed order).
//
// tower(x) = normalise(W2 . relu(W1 . x + b1) + b2), FP32 master weights with
// BF16 working copies.  Each matrix product takes BF16 operands (rounded to
// nearest even) and accumulates in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16): the tower input, the weights, the hidden
// activation after ReLU and, backwards, the pre-activation gradients entering
// the weight and input products.  Bias, ReLU, normalisation, logits and
// softmax stay in FP32.
//
// Loss (Eq. 2 / Eq. 4 read query-anchored over all hubs, the positive inside
// the denominator): L = mean_i [logsumexp_h(s_ih) - s_i,y_i],
// s_ih = <e_q_i, e_h> / tau.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------- BF16 GEMM
// C[m][n] = sum_k A(m,k) * B(n,k) with A(m,k) = A[m*sam + k*sak] and
// B(n,k) = B[n*sbn + k*sbk] (bf16).  Epilogue: + bias[n]; optional ReLU;
// optional multiply by (mask[m*ldc+n] > 0); FP32 result to C and/or BF16 to Cb.
struct GemmArgs {
    const uint16_t *A;
    int64_t sam, sak;
    const uint16_t *B;
    int64_t sbn, sbk;
    int M, N, K;
    const float *bias;
    int relu;
    const float *mask;
    float *C;
    uint16_t *Cb;
    int ldc;
};

constexpr int GT = 64;   // tile
constexpr int GK = 32;   // k step: one 16x16x32 product per block

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g)
{
    __shared__ uint16_t As[GT][GK + 4];
    __shared__ uint16_t Bs[GT][GK + 4];
    const int t = threadIdx.x;
    const int w = t >> 6, lane = t & 63;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    v4f acc[4];
    for (int b = 0; b < 4; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        for (int e = t; e < GT * GK; e += 256) {
            int r = e / GK, kk = e % GK;
            int m = m0 + r, n = n0 + r, k = k0 + kk;
            As[r][kk] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0;
            Bs[r][kk] = (n < g.N && k < g.K) ? g.B[(int64_t)n * g.sbn + (int64_t)k * g.sbk] : 0;
        }
        __syncthreads();
        // each lane: eight consecutive k of its row (A) and column (B); the
        // same k for both operands, so the products are those of the sum
        v8s a;
        const int ar = 16 * w + (lane & 15), kq = 8 * (lane >> 4);
        for (int q = 0; q < 8; ++q) a[q] = (short)As[ar][kq + q];
        for (int b = 0; b < 4; ++b) {
            v8s bv;
            const int bc = 16 * b + (lane & 15);
            for (int q = 0; q < 8; ++q) bv[q] = (short)Bs[bc][kq + q];
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                             __builtin_bit_cast(v8bf, bv), acc[b],
                                                             0, 0, 0);
        }
        __syncthreads();
    }
    for (int b = 0; b < 4; ++b) {
        const int n = n0 + 16 * b + (lane & 15);
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + 16 * w + 4 * (lane >> 4) + i;
            if (m >= g.M || n >= g.N) continue;
            float v = acc[b][i];
            if (g.bias) v += g.bias[n];
            if (g.relu) v = v > 0.f ? v : 0.f;
            const int64_t o = (int64_t)m * g.ldc + n;
            if (g.mask && !(g.mask[o] > 0.f)) v = 0.f;
            if (g.C) g.C[o] = v;
            if (g.Cb) g.Cb[o] = f2bf(v);
        }
    }
}

// ---------------------------------------------------------------- FP32 GEMM
// C[m][n] = alpha * sum_k A(m,k) * B(n,k), fixed k order per element.
struct GemmF {
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbn, sbk;
    int M, N, K;
    float alpha;
    float *C;
    int ldc;
};

__global__ void __launch_bounds__(256) gemm_f32_kernel(GemmF g)
{
    __shared__ float As[16][GT + 1];
    __shared__ float Bs[16][GT + 1];
    const int t = threadIdx.x;
    const int tr = (t / 16) * 4, tc = (t % 16) * 4;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        for (int e = t; e < 16 * GT; e += 256) {
            int kk = e / GT, r = e % GT;
            int m = m0 + r, n = n0 + r, k = k0 + kk;
            As[kk][r] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.f;
            Bs[kk][r] = (n < g.N && k < g.K) ? g.B[(int64_t)n * g.sbn + (int64_t)k * g.sbk] : 0.f;
        }
        __syncthreads();
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc + j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            int m = m0 + tr + i, n = n0 + tc + j;
            if (m < g.M && n < g.N) g.C[(int64_t)m * g.ldc + n] = g.alpha * acc[i][j];
        }
}

// ---------------------------------------------------------------- elementwise
__global__ void to_bf16_kernel(const float *x, int64_t count, uint16_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(x[i]);
}

// rows idx[i] of x (ld cols), times `scale`, -> bf16 rows i; idx NULL = identity
__global__ void gather_bf16_kernel(const float *x, int cols, const int32_t *idx, int rows,
                                   float scale, uint16_t *out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)rows * cols;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e / cols, c = e % cols;
        int64_t src = idx ? idx[r] : r;
        out[e] = f2bf(x[src * cols + c] * scale);
    }
}

// hub tower input [x_hub * vec_scale | features]: rows of base (hub ids) then the features
__global__ void hub_input_kernel(const float *base, int dim, const int32_t *hub_ids,
                                 const float *feat, int nfeat, int nh, float vec_scale,
                                 float *out32, uint16_t *outb)
{
    const int cols = dim + nfeat;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)nh * cols;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e / cols, c = e % cols;
        float v = c < dim ? base[(int64_t)hub_ids[r] * dim + c] * vec_scale
                          : feat[r * nfeat + (c - dim)];
        if (out32) out32[e] = v;
        if (outb) outb[e] = f2bf(v);
    }
}

// ------------------------------------------------- fused inference forward
// The forward of one tower for inference (no intermediates kept), one
// wavefront per 16 rows: x * in_scale rounded to BF16, the first product
// with bias and ReLU rounded to BF16 into LDS, the second product with bias,
// and the per-row normalisation.  Every step is the arithmetic of the
// training forward in the same order: the same operand rounding, the same
// lane layout and sequence of 32-deep MFMA steps per output element (the
// generic GEMM's), and the normalisation's sums and shuffles of
// normalise_kernel, so the embeddings are the same bits.
// HB = hidden / 16, DB = dout / 16; din % 8 == 0.
struct TowerInfer {
    const float *x;
    const int32_t *idx;   // row i of the input is x row idx[i] (NULL: row i)
    int rows, din;
    float scale;
    const uint16_t *W1b;
    const float *b1;
    const uint16_t *W2b;
    const float *b2;
    float *out;
};

template <int HB, int DB>
__global__ void __launch_bounds__(64) tower_infer_kernel(TowerInfer a)
{
    constexpr int HID = 16 * HB, DOUT = 16 * DB;
    __shared__ __align__(16) uint16_t H[16][HID + 8];
    __shared__ float Z[16][DOUT + 1];
    const int lane = threadIdx.x;
    const int rl = lane & 15, kq = 8 * (lane >> 4), rq = 4 * (lane >> 4);
    const int r0 = blockIdx.x * 16;
    const int row = r0 + rl;
    const bool live = row < a.rows;
    const float *xr = a.x + (live ? (int64_t)(a.idx ? a.idx[row] : row) * a.din : 0);
    v4f acc[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < a.din; k0 += 32) {
        const int k = k0 + kq;
        v8s av;
        if (live && k < a.din) {
            const float4 lo = *reinterpret_cast<const float4 *>(xr + k);
            const float4 hi = *reinterpret_cast<const float4 *>(xr + k + 4);
            av[0] = (short)f2bf(lo.x * a.scale);
            av[1] = (short)f2bf(lo.y * a.scale);
            av[2] = (short)f2bf(lo.z * a.scale);
            av[3] = (short)f2bf(lo.w * a.scale);
            av[4] = (short)f2bf(hi.x * a.scale);
            av[5] = (short)f2bf(hi.y * a.scale);
            av[6] = (short)f2bf(hi.z * a.scale);
            av[7] = (short)f2bf(hi.w * a.scale);
        } else {
            av = v8s{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int b = 0; b < HB; ++b) {
            const v8s bv = k < a.din
                               ? *reinterpret_cast<const v8s *>(a.W1b + (size_t)(16 * b + rl) * a.din + k)
                               : v8s{0, 0, 0, 0, 0, 0, 0, 0};
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av),
                                                             __builtin_bit_cast(v8bf, bv), acc[b],
                                                             0, 0, 0);
        }
    }
#pragma unroll
    for (int b = 0; b < HB; ++b) {
        const int n = 16 * b + rl;
        const float bias = a.b1[n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = acc[b][i] + bias;
            v = v > 0.f ? v : 0.f;
            H[rq + i][n] = f2bf(v);
        }
    }
    __syncthreads();
    v4f acc2[DB];
#pragma unroll
    for (int b = 0; b < DB; ++b) acc2[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < HID; k0 += 32) {
        const v8s av = *reinterpret_cast<const v8s *>(&H[rl][k0 + kq]);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const v8s bv = *reinterpret_cast<const v8s *>(a.W2b + (size_t)(16 * b + rl) * HID + k0 + kq);
            acc2[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av),
                                                              __builtin_bit_cast(v8bf, bv), acc2[b],
                                                              0, 0, 0);
        }
    }
#pragma unroll
    for (int b = 0; b < DB; ++b) {
        const int n = 16 * b + rl;
        const float bias = a.b2[n];
#pragma unroll
        for (int i = 0; i < 4; ++i) Z[rq + i][n] = acc2[b][i] + bias;
    }
    __syncthreads();
    // normalise_kernel's arithmetic, one row at a time
    for (int r = 0; r < 16 && r0 + r < a.rows; ++r) {
        float s = 0.f;
        for (int c = lane; c < DOUT; c += 64) s += Z[r][c] * Z[r][c];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        const float nrm = sqrtf(s);
        for (int c = lane; c < DOUT; c += 64) a.out[(int64_t)(r0 + r) * DOUT + c] = Z[r][c] / nrm;
    }
}

template <int HB>
bool launch_infer_d(const TowerInfer &a, int dout, hipStream_t st)
{
    const dim3 grid((unsigned)((a.rows + 15) / 16));
    switch (dout) {
    case 32: hipLaunchKernelGGL((tower_infer_kernel<HB, 2>), grid, dim3(64), 0, st, a); return true;
    case 64: hipLaunchKernelGGL((tower_infer_kernel<HB, 4>), grid, dim3(64), 0, st, a); return true;
    case 128: hipLaunchKernelGGL((tower_infer_kernel<HB, 8>), grid, dim3(64), 0, st, a); return true;
    default: return false;
    }
}

// launches the fused forward when the shapes and alignments allow it
bool tower_infer(const ann_tower &w, const float *x, const int32_t *idx, int rows, float *out,
                 hipStream_t st)
{
    if (w.din < 8 || w.din % 8 || !aligned(x, 16) || !aligned(w.W1b, 16) || !aligned(w.W2b, 16))
        return false;
    const TowerInfer a{x, idx, rows, w.din, w.in_scale, w.W1b, w.b1, w.W2b, w.b2, out};
    switch (w.hidden) {
    case 64: return launch_infer_d<4>(a, w.dout, st);
    case 128: return launch_infer_d<8>(a, w.dout, st);
    case 256: return launch_infer_d<16>(a, w.dout, st);
    default: return false;
    }
}

// one wavefront per row: e = z / |z|, keeps |z|
__global__ void normalise_kernel(const float *z, int rows, int cols, float *e, float *nrm)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    float s = 0.f;
    for (int c = lane; c < cols; c += 64) s += z[r * cols + c] * z[r * cols + c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const float n = sqrtf(s);
    for (int c = lane; c < cols; c += 64) e[r * cols + c] = z[r * cols + c] / n;
    if (lane == 0 && nrm) nrm[r] = n;
}

// dz = (de - e <e, de>) / |z|; also BF16 copy
__global__ void normalise_bwd_kernel(const float *e, const float *de, const float *nrm, int rows,
                                     int cols, float *dz, uint16_t *dzb)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    float s = 0.f;
    for (int c = lane; c < cols; c += 64) s += e[r * cols + c] * de[r * cols + c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    for (int c = lane; c < cols; c += 64) {
        float v = (de[r * cols + c] - e[r * cols + c] * s) / nrm[r];
        dz[r * cols + c] = v;
        dzb[r * cols + c] = f2bf(v);
    }
}

// one wavefront per query row of logits: loss_i and ds = (softmax - onehot)/B
__global__ void softmax_ce_kernel(const float *s, int rows, int cols, const int32_t *labels,
                                  const int32_t *idx, float inv_b, float *ds, float *loss_rows)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    const float *row = s + r * cols;
    float mx = -__int_as_float(0x7f800000);
    for (int c = lane; c < cols; c += 64) mx = fmaxf(mx, row[c]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float se = 0.f;
    for (int c = lane; c < cols; c += 64) se += expf(row[c] - mx);
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o);
    const int y = labels[idx ? idx[r] : r];
    for (int c = lane; c < cols; c += 64) {
        float p = expf(row[c] - mx) / se;
        ds[r * cols + c] = (p - (c == y ? 1.f : 0.f)) * inv_b;
    }
    if (lane == 0) loss_rows[r] = logf(se) + mx - row[y];
}

// Eq. 4 read hub-anchored: row i of s (Bh rows of `cols` scores) owns the
// block of W = P + N columns starting at i * W, its P positives then its N
// negatives.  One wavefront per hub row: loss_i = P * LSE_i - sum_pos s and
// ds = (P * softmax - [positive]) * inv_b inside the block, 0 elsewhere.
__global__ void hub_ce_kernel(const float *s, int rows, int cols, int P, int N, float inv_b,
                              float *ds, float *loss_rows)
{
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    const int W = P + N;
    const float *row = s + r * cols + r * W;
    float mx = -__int_as_float(0x7f800000);
    for (int c = lane; c < W; c += 64) mx = fmaxf(mx, row[c]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float se = 0.f, sp = 0.f;
    for (int c = lane; c < W; c += 64) {
        se += expf(row[c] - mx);
        if (c < P) sp += row[c];
    }
    for (int o = 32; o > 0; o >>= 1) {
        se += __shfl_xor(se, o);
        sp += __shfl_xor(sp, o);
    }
    float *drow = ds + r * cols;
    for (int c = lane; c < cols; c += 64) {
        const int j = c - (int)(r * W);
        float g = 0.f;
        if (j >= 0 && j < W) g = ((float)P * expf(row[j] - mx) / se - (j < P ? 1.f : 0.f)) * inv_b;
        drow[c] = g;
    }
    if (lane == 0) loss_rows[r] = (float)P * (logf(se) + mx) - sp;
}

// Column sums of x [rows x cols], each summed row by row in order (the
// training's bits depend on it); the loads of 16 rows are issued together
// before their adds, so the chain waits on memory once per 16 rows.
__global__ void bias_grad_kernel(const float *x, int rows, int cols, float *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    int r = 0;
    for (; r + 16 <= rows; r += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = x[(int64_t)(r + u) * cols + c];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; r < rows; ++r) s += x[(int64_t)r * cols + c];
    out[c] = s;
}

__global__ void mean_kernel(const float *x, int count, float *out)
{
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < count; i += 256) s += x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] / (float)count;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                            float b1, float b2, float eps, float c1, float c2, uint16_t *pb)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.f - b1) * gi;
        float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float mh = mi / c1, vh = vi / c2;
        float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

__global__ void scale_kernel(float *x, int64_t count, float a)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= a;
}

inline dim3 grid2(int M, int N) { return dim3((N + GT - 1) / GT, (M + GT - 1) / GT); }
inline int gridn(int64_t n) { return (int)((n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256); }

ann_status gemm_bf16(const GemmArgs &g, hipStream_t st)
{
    hipLaunchKernelGGL(gemm_bf16_kernel, grid2(g.M, g.N), dim3(256), 0, st, g);
    ANN_LAUNCHED();
    return ANN_OK;
}

ann_status gemm_f32(const GemmF &g, hipStream_t st)
{
    hipLaunchKernelGGL(gemm_f32_kernel, grid2(g.M, g.N), dim3(256), 0, st, g);
    ANN_LAUNCHED();
    return ANN_OK;
}

#define TRY(x)                              \
    do {                                    \
        ann_status s_ = (x);                \
        if (s_ != ANN_OK) return s_;        \
    } while (0)

// scratch of one tower pass over `rows` rows
struct TowerBufs {
    uint16_t *xb;    // rows x din
    float *z1;       // rows x hidden
    uint16_t *a1b;   // rows x hidden
    float *z2;       // rows x dout
    float *e;        // rows x dout
    float *nrm;      // rows
    float *de;       // rows x dout
    float *dz2;      // rows x dout
    uint16_t *dz2b;
    float *dz1;      // rows x hidden
    uint16_t *dz1b;
};

size_t tower_bufs_bytes(int rows, int din, int hidden, int dout)
{
    size_t b = 0;
    b += round_up((size_t)rows * din * 2, 256);
    b += round_up((size_t)rows * hidden * 4, 256) + round_up((size_t)rows * hidden * 2, 256);
    b += round_up((size_t)rows * dout * 4, 256) * 2 + round_up((size_t)rows * 4, 256);
    b += round_up((size_t)rows * dout * 4, 256) * 2 + round_up((size_t)rows * dout * 2, 256);
    b += round_up((size_t)rows * hidden * 4, 256) + round_up((size_t)rows * hidden * 2, 256);
    return b;
}

TowerBufs carve_tower(Carve &cv, int rows, int din, int hidden, int dout)
{
    TowerBufs t;
    t.xb = cv.take<uint16_t>((size_t)rows * din);
    t.z1 = cv.take<float>((size_t)rows * hidden);
    t.a1b = cv.take<uint16_t>((size_t)rows * hidden);
    t.z2 = cv.take<float>((size_t)rows * dout);
    t.e = cv.take<float>((size_t)rows * dout);
    t.nrm = cv.take<float>((size_t)rows);
    t.de = cv.take<float>((size_t)rows * dout);
    t.dz2 = cv.take<float>((size_t)rows * dout);
    t.dz2b = cv.take<uint16_t>((size_t)rows * dout);
    t.dz1 = cv.take<float>((size_t)rows * hidden);
    t.dz1b = cv.take<uint16_t>((size_t)rows * hidden);
    return t;
}

// forward from xb (already BF16) to e
ann_status tower_fwd(const ann_tower &w, const TowerBufs &b, int rows, hipStream_t st)
{
    GemmArgs g{};
    g.A = b.xb;
    g.sam = w.din;
    g.sak = 1;
    g.B = w.W1b;
    g.sbn = w.din;
    g.sbk = 1;
    g.M = rows;
    g.N = w.hidden;
    g.K = w.din;
    g.bias = w.b1;
    g.relu = 1;
    g.C = b.z1;   // post-ReLU activation (its sign is the ReLU mask)
    g.Cb = b.a1b;
    g.ldc = w.hidden;
    TRY(gemm_bf16(g, st));
    GemmArgs h{};
    h.A = b.a1b;
    h.sam = w.hidden;
    h.sak = 1;
    h.B = w.W2b;
    h.sbn = w.hidden;
    h.sbk = 1;
    h.M = rows;
    h.N = w.dout;
    h.K = w.hidden;
    h.bias = w.b2;
    h.C = b.z2;
    h.ldc = w.dout;
    TRY(gemm_bf16(h, st));
    hipLaunchKernelGGL(normalise_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, b.z2, rows, w.dout,
                       b.e, b.nrm);
    ANN_LAUNCHED();
    return ANN_OK;
}

// backward from b.de; writes gradients into gr
ann_status tower_bwd(const ann_tower &w, const ann_tower_grads &gr, const TowerBufs &b, int rows,
                     hipStream_t st)
{
    hipLaunchKernelGGL(normalise_bwd_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, b.e, b.de,
                       b.nrm, rows, w.dout, b.dz2, b.dz2b);
    ANN_LAUNCHED();
    // dW2 [dout x hidden] = dz2b^T . a1b
    GemmArgs g{};
    g.A = b.dz2b;
    g.sam = 1;
    g.sak = w.dout;
    g.B = b.a1b;
    g.sbn = 1;
    g.sbk = w.hidden;
    g.M = w.dout;
    g.N = w.hidden;
    g.K = rows;
    g.C = gr.gW2;
    g.ldc = w.hidden;
    TRY(gemm_bf16(g, st));
    hipLaunchKernelGGL(bias_grad_kernel, dim3((w.dout + 255) / 256), dim3(256), 0, st, b.dz2, rows,
                       w.dout, gr.gb2);
    ANN_LAUNCHED();
    // dz1 [rows x hidden] = (dz2b . W2b) * (z1 > 0)
    GemmArgs h{};
    h.A = b.dz2b;
    h.sam = w.dout;
    h.sak = 1;
    h.B = w.W2b;
    h.sbn = 1;
    h.sbk = w.hidden;
    h.M = rows;
    h.N = w.hidden;
    h.K = w.dout;
    h.mask = b.z1;
    h.C = b.dz1;
    h.Cb = b.dz1b;
    h.ldc = w.hidden;
    TRY(gemm_bf16(h, st));
    hipLaunchKernelGGL(bias_grad_kernel, dim3((w.hidden + 255) / 256), dim3(256), 0, st, b.dz1, rows,
                       w.hidden, gr.gb1);
    ANN_LAUNCHED();
    // dW1 [hidden x din] = dz1b^T . xb
    GemmArgs k{};
    k.A = b.dz1b;
    k.sam = 1;
    k.sak = w.hidden;
    k.B = b.xb;
    k.sbn = 1;
    k.sbk = w.din;
    k.M = w.hidden;
    k.N = w.din;
    k.K = rows;
    k.C = gr.gW1;
    k.ldc = w.din;
    TRY(gemm_bf16(k, st));
    return ANN_OK;
}

ann_status adam(ann_tower &w, const ann_tower_grads &gr, const ann_adam_state &a, int step,
                float lr, hipStream_t st)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    const int64_t n1 = (int64_t)w.hidden * w.din, n2 = (int64_t)w.dout * w.hidden;
    hipLaunchKernelGGL(adam_kernel, dim3(gridn(n1)), dim3(256), 0, st, w.W1, gr.gW1, a.mW1, a.vW1, n1,
                       lr, b1, b2, eps, c1, c2, w.W1b);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(adam_kernel, dim3(gridn(w.hidden)), dim3(256), 0, st, w.b1, gr.gb1, a.mb1,
                       a.vb1, (int64_t)w.hidden, lr, b1, b2, eps, c1, c2, (uint16_t *)nullptr);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(adam_kernel, dim3(gridn(n2)), dim3(256), 0, st, w.W2, gr.gW2, a.mW2, a.vW2, n2,
                       lr, b1, b2, eps, c1, c2, w.W2b);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(adam_kernel, dim3(gridn(w.dout)), dim3(256), 0, st, w.b2, gr.gb2, a.mb2,
                       a.vb2, (int64_t)w.dout, lr, b1, b2, eps, c1, c2, (uint16_t *)nullptr);
    ANN_LAUNCHED();
    return ANN_OK;
}

ann_status check_tower(const ann_tower *w, const char *name)
{
    ANN_REQUIRE(w != nullptr, "%s tower is NULL", name);
    ANN_REQUIRE(w->W1 && w->b1 && w->W2 && w->b2 && w->W1b && w->W2b, "%s tower has a NULL pointer",
                name);
    ANN_REQUIRE(w->din >= 1 && w->hidden >= 1 && w->dout >= 1, "%s tower has a bad shape", name);
    ANN_REQUIRE(w->in_scale > 0.f, "%s tower in_scale must be > 0", name);
    ANN_SUPPORTED(w->dout <= 1024 && w->hidden <= 4096 && w->din <= 4096, "%s tower too large",
                  name);
    return ANN_OK;
}

}  // namespace

size_t tower_forward_ws(int rows, const ann_tower *w)
{
    return tower_bufs_bytes(rows, w->din, w->hidden, w->dout) + 256;
}

size_t train_step_ws(int batch, int nh, int din_q, int din_h, int hidden, int dout)
{
    size_t b = tower_bufs_bytes(batch, din_q, hidden, dout) + tower_bufs_bytes(nh, din_h, hidden, dout);
    b += round_up((size_t)batch * nh * 4, 256) * 2;    // logits, dlogits
    b += round_up((size_t)batch * 4, 256) + 1024;
    return b;
}

size_t train_hub_ws(int bh, int P, int N, int din_q, int din_h, int hidden, int dout)
{
    const int rows = bh * (P + N);
    size_t b = tower_bufs_bytes(rows, din_q, hidden, dout) + tower_bufs_bytes(bh, din_h, hidden, dout);
    b += round_up((size_t)bh * rows * 4, 256) * 2;     // scores, their gradient
    b += round_up((size_t)bh * 4, 256) + 1024;
    return b;
}

// forward of one tower over rows of x (FP32, rows x din) -> unit embeddings
ann_status tower_forward_run(const ann_tower &w, const float *x, const int32_t *idx, int rows,
                             float *out, void *ws, hipStream_t st)
{
    if (rows > 0 && tower_infer(w, x, idx, rows, out, st)) {
        ANN_LAUNCHED();
        return ANN_OK;
    }
    Carve cv{static_cast<unsigned char *>(ws)};
    TowerBufs b = carve_tower(cv, rows, w.din, w.hidden, w.dout);
    b.e = out;
    hipLaunchKernelGGL(gather_bf16_kernel, dim3(gridn((int64_t)rows * w.din)), dim3(256), 0, st, x,
                       w.din, idx, rows, w.in_scale, b.xb);
    ANN_LAUNCHED();
    return tower_fwd(w, b, rows, st);
}

ann_status refresh_bf16(const ann_tower &w, hipStream_t st)
{
    const int64_t n1 = (int64_t)w.hidden * w.din, n2 = (int64_t)w.dout * w.hidden;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(gridn(n1)), dim3(256), 0, st, w.W1, n1, w.W1b);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(to_bf16_kernel, dim3(gridn(n2)), dim3(256), 0, st, w.W2, n2, w.W2b);
    ANN_LAUNCHED();
    return ANN_OK;
}

}  // namespace ann

using namespace ann;

extern "C" ann_status ann_hub_input(const float *base, int64_t n, int32_t dim, const int32_t *hub_ids,
                                    int32_t n_hubs, const float *features, int32_t n_feat,
                                    float vec_scale, float *out, void *stream)
{
    ANN_REQUIRE(base && hub_ids && out, "a required pointer is NULL");
    ANN_REQUIRE(n_feat == 0 || features, "features is NULL");
    ANN_REQUIRE(n >= 1 && dim >= 1 && n_hubs >= 1 && n_feat >= 0, "bad sizes");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t count = (int64_t)n_hubs * (dim + n_feat);
    hipLaunchKernelGGL(hub_input_kernel, dim3(gridn(count)), dim3(256), 0, st, base, dim, hub_ids,
                       features, n_feat, n_hubs, vec_scale, out, (uint16_t *)nullptr);
    ANN_LAUNCHED();
    return ANN_OK;
}

extern "C" size_t ann_tower_workspace_size(const ann_tower *tower, int32_t rows)
{
    return tower ? tower_forward_ws(rows, tower) : 0;
}

extern "C" size_t ann_train_workspace_size(int32_t batch, int32_t n_hubs, int32_t din_q,
                                           int32_t din_h, int32_t hidden, int32_t dout)
{
    return train_step_ws(batch, n_hubs, din_q, din_h, hidden, dout);
}

extern "C" ann_status ann_tower_sync(const ann_tower *tower, void *stream)
{
    ann_status s = check_tower(tower, "the");
    if (s != ANN_OK) return s;
    return refresh_bf16(*tower, static_cast<hipStream_t>(stream));
}

extern "C" ann_status ann_tower_forward(const ann_tower *tower, const float *x, int32_t rows,
                                        float *out, void *workspace, size_t ws_bytes, void *stream)
{
    ann_status s = check_tower(tower, "the");
    if (s != ANN_OK) return s;
    ANN_REQUIRE(rows >= 0, "rows must be >= 0");
    ANN_REQUIRE(rows == 0 || (x && out && workspace), "a required pointer is NULL");
    ANN_REQUIRE(ws_bytes >= tower_forward_ws(rows, tower), "workspace too small");
    if (rows == 0) return ANN_OK;
    return tower_forward_run(*tower, x, nullptr, rows, out, workspace,
                             static_cast<hipStream_t>(stream));
}

extern "C" ann_status ann_train_step(ann_tower *qt, ann_tower *ht, const ann_tower_grads *qg,
                                     const ann_tower_grads *hg, const ann_adam_state *qa,
                                     const ann_adam_state *ha, const float *train_q,
                                     const int32_t *batch_idx, int32_t batch,
                                     const int32_t *labels, const float *hub_in, int32_t n_hubs,
                                     float tau, float lr, int32_t step, float *loss,
                                     float *q_emb, float *h_emb, float *hub_in_grad,
                                     void *workspace, size_t ws_bytes, void *stream)
{
    ann_status s = check_tower(qt, "query");
    if (s != ANN_OK) return s;
    s = check_tower(ht, "hub");
    if (s != ANN_OK) return s;
    ANN_REQUIRE(qg && hg, "gradient buffers are NULL");
    ANN_REQUIRE(qg->gW1 && qg->gb1 && qg->gW2 && qg->gb2 && hg->gW1 && hg->gb1 && hg->gW2 && hg->gb2,
                "a gradient pointer is NULL");
    ANN_REQUIRE(train_q && labels && hub_in && loss && workspace, "a required pointer is NULL");
    ANN_REQUIRE(batch >= 1 && n_hubs >= 1, "batch and n_hubs must be >= 1");
    ANN_REQUIRE(qt->dout == ht->dout && qt->hidden == ht->hidden,
                "towers must share hidden and output sizes");
    ANN_REQUIRE(tau > 0.f, "tau must be > 0");
    ANN_REQUIRE(step >= 0, "step must be >= 0");
    ANN_REQUIRE(step == 0 || (qa && ha), "Adam state needed when step > 0");
    ANN_REQUIRE(ws_bytes >= train_step_ws(batch, n_hubs, qt->din, ht->din, qt->hidden, qt->dout),
                "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Carve cv{static_cast<unsigned char *>(workspace)};
    TowerBufs bq = carve_tower(cv, batch, qt->din, qt->hidden, qt->dout);
    TowerBufs bh = carve_tower(cv, n_hubs, ht->din, ht->hidden, ht->dout);
    float *logits = cv.take<float>((size_t)batch * n_hubs);
    float *dlog = cv.take<float>((size_t)batch * n_hubs);
    float *lrow = cv.take<float>((size_t)batch);
    if (q_emb) bq.e = q_emb;
    if (h_emb) bh.e = h_emb;

    // forward
    hipLaunchKernelGGL(gather_bf16_kernel, dim3(gridn((int64_t)batch * qt->din)), dim3(256), 0, st,
                       train_q, qt->din, batch_idx, batch, qt->in_scale, bq.xb);
    ANN_LAUNCHED();
    TRY(tower_fwd(*qt, bq, batch, st));
    hipLaunchKernelGGL(gather_bf16_kernel, dim3(gridn((int64_t)n_hubs * ht->din)), dim3(256), 0, st,
                       hub_in, ht->din, (const int32_t *)nullptr, n_hubs, ht->in_scale, bh.xb);
    ANN_LAUNCHED();
    TRY(tower_fwd(*ht, bh, n_hubs, st));
    const int e = qt->dout;
    GemmF lg{bq.e, e, 1, bh.e, e, 1, batch, n_hubs, e, 1.f / tau, logits, n_hubs};
    TRY(gemm_f32(lg, st));
    hipLaunchKernelGGL(softmax_ce_kernel, dim3((batch + 3) / 4), dim3(256), 0, st, logits, batch,
                       n_hubs, labels, batch_idx, 1.f / (float)batch, dlog, lrow);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, lrow, batch, loss);
    ANN_LAUNCHED();
    // dEq [batch x e] = dlog . Eh / tau ; dEh [nh x e] = dlog^T . Eq / tau
    GemmF gq{dlog, n_hubs, 1, bh.e, 1, e, batch, e, n_hubs, 1.f / tau, bq.de, e};
    TRY(gemm_f32(gq, st));
    GemmF gh{dlog, 1, n_hubs, bq.e, 1, e, n_hubs, e, batch, 1.f / tau, bh.de, e};
    TRY(gemm_f32(gh, st));
    TRY(tower_bwd(*qt, *qg, bq, batch, st));
    TRY(tower_bwd(*ht, *hg, bh, n_hubs, st));
    if (hub_in_grad) {
        // dL/d hub_in [n_hubs x din_h] = in_scale * (dz1b . W1b)
        GemmArgs g{};
        g.A = bh.dz1b;
        g.sam = ht->hidden;
        g.sak = 1;
        g.B = ht->W1b;
        g.sbn = 1;
        g.sbk = ht->din;
        g.M = n_hubs;
        g.N = ht->din;
        g.K = ht->hidden;
        g.C = hub_in_grad;
        g.ldc = ht->din;
        TRY(gemm_bf16(g, st));
        if (ht->in_scale != 1.f) {
            const int64_t cnt = (int64_t)n_hubs * ht->din;
            hipLaunchKernelGGL(scale_kernel, dim3(gridn(cnt)), dim3(256), 0, st, hub_in_grad, cnt,
                               ht->in_scale);
            ANN_LAUNCHED();
        }
    }
    if (step > 0) {
        TRY(adam(*qt, *qg, *qa, step, lr, st));
        TRY(adam(*ht, *hg, *ha, step, lr, st));
    }
    return ANN_OK;
}

extern "C" size_t ann_train_hub_workspace_size(int32_t hubs, int32_t P, int32_t N, int32_t din_q,
                                               int32_t din_h, int32_t hidden, int32_t dout)
{
    if (hubs < 1 || P < 1 || N < 0) return 0;
    return train_hub_ws(hubs, P, N, din_q, din_h, hidden, dout);
}

extern "C" ann_status ann_train_step_hub(ann_tower *qt, ann_tower *ht, const ann_tower_grads *qg,
                                         const ann_tower_grads *hg, const ann_adam_state *qa,
                                         const ann_adam_state *ha, const float *train_q,
                                         const int32_t *q_idx, const int32_t *hub_idx,
                                         int32_t hubs, int32_t P, int32_t N, const float *hub_in,
                                         float tau, float lr, int32_t step, float *loss,
                                         float *q_emb, float *h_emb, void *workspace,
                                         size_t ws_bytes, void *stream)
{
    ann_status s = check_tower(qt, "query");
    if (s != ANN_OK) return s;
    s = check_tower(ht, "hub");
    if (s != ANN_OK) return s;
    ANN_REQUIRE(qg && hg, "gradient buffers are NULL");
    ANN_REQUIRE(qg->gW1 && qg->gb1 && qg->gW2 && qg->gb2 && hg->gW1 && hg->gb1 && hg->gW2 && hg->gb2,
                "a gradient pointer is NULL");
    ANN_REQUIRE(train_q && q_idx && hub_idx && hub_in && loss && workspace,
                "a required pointer is NULL");
    ANN_REQUIRE(hubs >= 1 && P >= 1 && N >= 0, "need hubs >= 1, P >= 1, N >= 0");
    ANN_REQUIRE(qt->dout == ht->dout && qt->hidden == ht->hidden,
                "towers must share hidden and output sizes");
    ANN_REQUIRE(tau > 0.f, "tau must be > 0");
    ANN_REQUIRE(step >= 0, "step must be >= 0");
    ANN_REQUIRE(step == 0 || (qa && ha), "Adam state needed when step > 0");
    ANN_REQUIRE(ws_bytes >= train_hub_ws(hubs, P, N, qt->din, ht->din, qt->hidden, qt->dout),
                "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int rows = hubs * (P + N);
    Carve cv{static_cast<unsigned char *>(workspace)};
    TowerBufs bq = carve_tower(cv, rows, qt->din, qt->hidden, qt->dout);
    TowerBufs bh = carve_tower(cv, hubs, ht->din, ht->hidden, ht->dout);
    float *sc = cv.take<float>((size_t)hubs * rows);
    float *dsc = cv.take<float>((size_t)hubs * rows);
    float *lrow = cv.take<float>((size_t)hubs);
    if (q_emb) bq.e = q_emb;
    if (h_emb) bh.e = h_emb;

    // forward: the batch's queries and hubs through their towers
    hipLaunchKernelGGL(gather_bf16_kernel, dim3(gridn((int64_t)rows * qt->din)), dim3(256), 0, st,
                       train_q, qt->din, q_idx, rows, qt->in_scale, bq.xb);
    ANN_LAUNCHED();
    TRY(tower_fwd(*qt, bq, rows, st));
    hipLaunchKernelGGL(gather_bf16_kernel, dim3(gridn((int64_t)hubs * ht->din)), dim3(256), 0, st,
                       hub_in, ht->din, hub_idx, hubs, ht->in_scale, bh.xb);
    ANN_LAUNCHED();
    TRY(tower_fwd(*ht, bh, hubs, st));
    const int e = qt->dout;
    // scores [hubs x rows] = Eh . Eq^T / tau (only each hub's own block is used)
    GemmF lg{bh.e, e, 1, bq.e, e, 1, hubs, rows, e, 1.f / tau, sc, rows};
    TRY(gemm_f32(lg, st));
    hipLaunchKernelGGL(hub_ce_kernel, dim3((hubs + 3) / 4), dim3(256), 0, st, sc, hubs, rows, P, N,
                       1.f / (float)hubs, dsc, lrow);
    ANN_LAUNCHED();
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, lrow, hubs, loss);
    ANN_LAUNCHED();
    // dEh [hubs x e] = dS . Eq / tau ; dEq [rows x e] = dS^T . Eh / tau
    GemmF gh{dsc, rows, 1, bq.e, 1, e, hubs, e, rows, 1.f / tau, bh.de, e};
    TRY(gemm_f32(gh, st));
    GemmF gq{dsc, 1, rows, bh.e, 1, e, rows, e, hubs, 1.f / tau, bq.de, e};
    TRY(gemm_f32(gq, st));
    TRY(tower_bwd(*qt, *qg, bq, rows, st));
    TRY(tower_bwd(*ht, *hg, bh, hubs, st));
    if (step > 0) {
        TRY(adam(*qt, *qg, *qa, step, lr, st));
        TRY(adam(*ht, *hg, *ha, step, lr, st));
    }
    return ANN_OK;
}
