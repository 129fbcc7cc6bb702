// Fusion embedding augmentation (Eq. 3): multi-head attention of a hub's
// vector p over its topology tokens U (S tokens of du values; masked slots
// are absent):
//   q = p WQ^T, K_s = U_s WK^T, V_s = U_s WV^T          (m heads of dk channels)
//   a_j = softmax_s( <q_j, K_s,j> / sqrt(dk) )           over present tokens
//   F = concat_j( sum_s a_j,s V_s,j ) WO^T
// A hub without tokens gets F = 0.  FP32 throughout; one 64-thread block per
// hub (channel t of the m*dk <= 64 on thread t), every sum in a fixed order,
// and the backward pass writes per-hub partial gradients that a second kernel
// sums in hub order, so results do not depend on scheduling.
#include "common.h"
#include "internal.h"

namespace ann {
namespace {

constexpr int FU_MAXC = 64;   // m * dk, dF and S are at most 64
constexpr int FU_MAXH = 16;   // heads

struct FusionArgs {
    const float *WQ, *WK, *WV, *WO;   // [C x dp], [C x du], [C x du], [dF x C]
    int heads, dk, dp, du, df, S, nh;
    const float *p;                   // nh x dp
    const float *U;                   // nh x S x du
    const uint8_t *mask;              // nh x S
};

// q, K, V, attention weights and the per-head outputs of hub i in LDS
struct FuState {
    float q[FU_MAXC];
    float K[FU_MAXC][FU_MAXC + 1];
    float V[FU_MAXC][FU_MAXC + 1];
    float a[FU_MAXH][FU_MAXC];        // [head][token]
    float O[FU_MAXC];
};

__device__ void fu_attend(const FusionArgs &f, int i, FuState &s)
{
    const int t = threadIdx.x;
    const int C = f.heads * f.dk;
    const float *pi = f.p + (int64_t)i * f.dp;
    const float *Ui = f.U + (int64_t)i * f.S * f.du;
    const uint8_t *mi = f.mask + (int64_t)i * f.S;
    if (t < C) {
        float acc = 0.f;
        for (int c = 0; c < f.dp; ++c) acc += pi[c] * f.WQ[(int64_t)t * f.dp + c];
        s.q[t] = acc;
        for (int u = 0; u < f.S; ++u) {
            float k = 0.f, v = 0.f;
            const float *Us = Ui + (int64_t)u * f.du;
            for (int c = 0; c < f.du; ++c) {
                k += Us[c] * f.WK[(int64_t)t * f.du + c];
                v += Us[c] * f.WV[(int64_t)t * f.du + c];
            }
            s.K[u][t] = k;
            s.V[u][t] = v;
        }
    }
    __syncthreads();
    // head j (thread j): scores, masked softmax in token order
    if (t < f.heads) {
        const float inv = 1.f / sqrtf((float)f.dk);
        float mx = -__int_as_float(0x7f800000);
        for (int u = 0; u < f.S; ++u) {
            float sc = 0.f;
            for (int c = t * f.dk; c < (t + 1) * f.dk; ++c) sc += s.q[c] * s.K[u][c];
            sc *= inv;
            s.a[t][u] = sc;
            if (mi[u] && sc > mx) mx = sc;
        }
        float sum = 0.f;
        for (int u = 0; u < f.S; ++u) {
            const float e = mi[u] ? expf(s.a[t][u] - mx) : 0.f;
            s.a[t][u] = e;
            sum += e;
        }
        for (int u = 0; u < f.S; ++u) s.a[t][u] = sum > 0.f ? s.a[t][u] / sum : 0.f;
    }
    __syncthreads();
    if (t < C) {
        const int j = t / f.dk;
        float o = 0.f;
        for (int u = 0; u < f.S; ++u) o += s.a[j][u] * s.V[u][t];
        s.O[t] = o;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(64) fusion_fwd_kernel(FusionArgs f, float *F)
{
    __shared__ FuState s;
    const int i = blockIdx.x;
    fu_attend(f, i, s);
    const int t = threadIdx.x;
    const int C = f.heads * f.dk;
    if (t < f.df) {
        float acc = 0.f;
        for (int c = 0; c < C; ++c) acc += s.O[c] * f.WO[(int64_t)t * C + c];
        F[(int64_t)i * f.df + t] = acc;
    }
}

// per-hub partial gradients: part + i * stride holds [gWQ | gWK | gWV | gWO]
__global__ void __launch_bounds__(64) fusion_bwd_kernel(FusionArgs f, const float *dF, float *part,
                                                        int64_t stride)
{
    __shared__ FuState s;
    __shared__ float dO[FU_MAXC], dq[FU_MAXC], ds[FU_MAXH][FU_MAXC];
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    const int C = f.heads * f.dk;
    fu_attend(f, i, s);
    const float *dFi = dF + (int64_t)i * f.df;
    float *gQ = part + (int64_t)i * stride;
    float *gK = gQ + (int64_t)C * f.dp;
    float *gV = gK + (int64_t)C * f.du;
    float *gO = gV + (int64_t)C * f.du;
    if (t < C) {
        float acc = 0.f;
        for (int o = 0; o < f.df; ++o) acc += dFi[o] * f.WO[(int64_t)o * C + t];
        dO[t] = acc;
    }
    if (t < f.df)
        for (int c = 0; c < C; ++c) gO[(int64_t)t * C + c] = dFi[t] * s.O[c];
    __syncthreads();
    // head j (thread j): da_u = <dO_j, V_u,j>, then the softmax backward
    if (t < f.heads) {
        float dot = 0.f;
        for (int u = 0; u < f.S; ++u) {
            float da = 0.f;
            for (int c = t * f.dk; c < (t + 1) * f.dk; ++c) da += dO[c] * s.V[u][c];
            ds[t][u] = da;
            dot += s.a[t][u] * da;
        }
        for (int u = 0; u < f.S; ++u) ds[t][u] = s.a[t][u] * (ds[t][u] - dot);
    }
    __syncthreads();
    const float inv = 1.f / sqrtf((float)f.dk);
    if (t < C) {
        const int j = t / f.dk;
        float acc = 0.f;
        for (int u = 0; u < f.S; ++u) acc += ds[j][u] * s.K[u][t];
        dq[t] = acc * inv;
    }
    __syncthreads();
    // dK_u,t = ds_j,u q_t / sqrt(dk) and dV_u,t = a_j,u dO_t, so
    // gWK[t][c] = q_t / sqrt(dk) sum_u ds_j,u U_u,c and gWV[t][c] = dO_t sum_u a_j,u U_u,c
    const float *pi = f.p + (int64_t)i * f.dp;
    const float *Ui = f.U + (int64_t)i * f.S * f.du;
    if (t < C) {
        const int j = t / f.dk;
        for (int c = 0; c < f.dp; ++c) gQ[(int64_t)t * f.dp + c] = dq[t] * pi[c];
        for (int c = 0; c < f.du; ++c) {
            float k = 0.f, v = 0.f;
            for (int u = 0; u < f.S; ++u) {
                const float x = Ui[(int64_t)u * f.du + c];
                k += ds[j][u] * x;
                v += s.a[j][u] * x;
            }
            gK[(int64_t)t * f.du + c] = s.q[t] * inv * k;
            gV[(int64_t)t * f.du + c] = dO[t] * v;
        }
    }
}

// out[e] = sum over hubs (in order) of part[i * stride + e]
__global__ void fusion_reduce_kernel(const float *part, int nh, int64_t stride, float *gQ, float *gK,
                                     float *gV, float *gO, int64_t nQ, int64_t nK, int64_t nO)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < stride;
         e += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int i = 0; i < nh; ++i) acc += part[(int64_t)i * stride + e];
        if (e < nQ) gQ[e] = acc;
        else if (e < nQ + nK) gK[e - nQ] = acc;
        else if (e < nQ + 2 * nK) gV[e - nQ - nK] = acc;
        else gO[e - nQ - 2 * nK] = acc;
    }
}

__global__ void adam_plain_kernel(float *p, const float *g, float *m, float *v, int64_t count,
                                  float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

int64_t fu_stride(const ann_fusion &f)
{
    const int64_t C = (int64_t)f.heads * f.dk;
    return C * f.dp + 2 * C * f.du + (int64_t)f.df * C;
}

ann_status fu_check(const ann_fusion *f, int nh, int S)
{
    ANN_REQUIRE(f != nullptr, "fusion is NULL");
    ANN_REQUIRE(f->WQ && f->WK && f->WV && f->WO, "a fusion matrix is NULL");
    ANN_REQUIRE(f->heads >= 1 && f->heads <= FU_MAXH && f->dk >= 1 && f->heads * f->dk <= FU_MAXC,
                "need 1 <= heads <= 16 and heads * dk <= 64");
    ANN_REQUIRE(f->df >= 1 && f->df <= FU_MAXC, "df must be in [1, 64]");
    ANN_REQUIRE(f->dp >= 1 && f->du >= 1, "dp and du must be >= 1");
    ANN_REQUIRE(S >= 1 && S <= FU_MAXC, "S must be in [1, 64]");
    ANN_REQUIRE(nh >= 0, "n_hubs must be >= 0");
    return ANN_OK;
}

FusionArgs fu_args(const ann_fusion &f, const float *p, const float *U, const uint8_t *mask, int nh,
                   int S)
{
    FusionArgs a{};
    a.WQ = f.WQ;
    a.WK = f.WK;
    a.WV = f.WV;
    a.WO = f.WO;
    a.heads = f.heads;
    a.dk = f.dk;
    a.dp = f.dp;
    a.du = f.du;
    a.df = f.df;
    a.S = S;
    a.nh = nh;
    a.p = p;
    a.U = U;
    a.mask = mask;
    return a;
}

// Tokens of the fusion embedding for hub c (one workgroup per hub): its
// vector p = x_hub * scale and, per graph slot s, U_s = (x_w - x_hub) * scale
// for the neighbour w in that slot (0 and mask 0 for an empty slot).
__global__ void __launch_bounds__(256) fusion_tokens_kernel(const float *base, int dim,
                                                            const int32_t *graph, int R,
                                                            const int32_t *hub_ids, float scale,
                                                            float *p, float *U, uint8_t *mask)
{
    const int c = blockIdx.x;
    const int64_t hub = hub_ids[c];
    const float *xh = base + hub * dim;
    for (int j = threadIdx.x; j < dim; j += blockDim.x) p[(int64_t)c * dim + j] = xh[j] * scale;
    for (int s = 0; s < R; ++s) {
        const int32_t w = graph[hub * R + s];
        float *u = U + ((int64_t)c * R + s) * dim;
        if (threadIdx.x == 0) mask[(int64_t)c * R + s] = w >= 0 ? 1 : 0;
        if (w < 0) {
            for (int j = threadIdx.x; j < dim; j += blockDim.x) u[j] = 0.f;
        } else {
            const float *xw = base + (int64_t)w * dim;
            for (int j = threadIdx.x; j < dim; j += blockDim.x) u[j] = (xw[j] - xh[j]) * scale;
        }
    }
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" ann_status ann_fusion_tokens(const float *base, int64_t n, int32_t dim,
                                        const int32_t *graph, int32_t R, const int32_t *hub_ids,
                                        int32_t n_hubs, float scale, float *p, float *U,
                                        uint8_t *mask, void *stream)
{
    ANN_REQUIRE(n >= 1 && dim >= 1 && R >= 1 && n_hubs >= 0, "need n, dim, R >= 1, n_hubs >= 0");
    if (n_hubs == 0) return ANN_OK;
    ANN_REQUIRE(base && graph && hub_ids && p && U && mask, "a required pointer is NULL");
    hipLaunchKernelGGL(fusion_tokens_kernel, dim3((unsigned)n_hubs), dim3(256), 0,
                       static_cast<hipStream_t>(stream), base, dim, graph, R, hub_ids, scale, p, U,
                       mask);
    ANN_LAUNCHED();
    return ANN_OK;
}

extern "C" size_t ann_fusion_workspace_size(const ann_fusion *f, int32_t n_hubs)
{
    if (!f || n_hubs < 0) return 0;
    return round_up((size_t)n_hubs * fu_stride(*f) * 4, 256) + 256;
}

extern "C" ann_status ann_fusion_forward(const ann_fusion *f, const float *p, const float *U,
                                         const uint8_t *mask, int32_t n_hubs, int32_t S, float *F,
                                         void *stream)
{
    ann_status s = fu_check(f, n_hubs, S);
    if (s != ANN_OK) return s;
    if (n_hubs == 0) return ANN_OK;
    ANN_REQUIRE(p && U && mask && F, "a required pointer is NULL");
    hipLaunchKernelGGL(fusion_fwd_kernel, dim3((unsigned)n_hubs), dim3(64), 0,
                       static_cast<hipStream_t>(stream), fu_args(*f, p, U, mask, n_hubs, S), F);
    ANN_LAUNCHED();
    return ANN_OK;
}

extern "C" ann_status ann_fusion_backward(const ann_fusion *f, const float *p, const float *U,
                                          const uint8_t *mask, int32_t n_hubs, int32_t S,
                                          const float *dF, float *gWQ, float *gWK, float *gWV,
                                          float *gWO, void *workspace, size_t ws_bytes, void *stream)
{
    ann_status s = fu_check(f, n_hubs, S);
    if (s != ANN_OK) return s;
    ANN_REQUIRE(gWQ && gWK && gWV && gWO, "a gradient pointer is NULL");
    ANN_REQUIRE(n_hubs == 0 || (p && U && mask && dF && workspace), "a required pointer is NULL");
    ANN_REQUIRE(ws_bytes >= ann_fusion_workspace_size(f, n_hubs), "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t stride = fu_stride(*f);
    const int64_t C = (int64_t)f->heads * f->dk;
    float *part = static_cast<float *>(workspace);
    if (n_hubs > 0) {
        hipLaunchKernelGGL(fusion_bwd_kernel, dim3((unsigned)n_hubs), dim3(64), 0, st,
                           fu_args(*f, p, U, mask, n_hubs, S), dF, part, stride);
        ANN_LAUNCHED();
    }
    int64_t blocks = (stride + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fusion_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, part, n_hubs,
                       stride, gWQ, gWK, gWV, gWO, C * f->dp, C * f->du, (int64_t)f->df * C);
    ANN_LAUNCHED();
    return ANN_OK;
}

extern "C" ann_status ann_adam_step(float *param, const float *grad, float *m, float *v,
                                    int64_t count, float lr, int32_t step, void *stream)
{
    ANN_REQUIRE(param && grad && m && v, "a required pointer is NULL");
    ANN_REQUIRE(count >= 0 && step >= 1, "need count >= 0 and step >= 1");
    if (count == 0) return ANN_OK;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(adam_plain_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), param, grad, m, v, count, lr, b1, b2, eps,
                       c1, c2);
    ANN_LAUNCHED();
    return ANN_OK;
}
