// Exact brute-force k nearest neighbours on the GPU (ground truth for
// recall, Eq. 1, and the candidate lists of the proximity graph).
//
// Two distance engines feed the shared top-K selection of knn_core.h:
//   * integer engine: every value is an integer in [0, 255]; vectors are
//     shifted by -128 into int8 and the dot products run on the int8 matrix
//     cores (v_mfma_i32_16x16x64_i8); d2 = |x'|^2 + |y'|^2 - 2 x'.y' is exact
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
// Values are integers in [0, 255], shifted by -128 into int8; d2 = |x'|^2 +
// |y'|^2 - 2 x'.y' is exact in int32 (below 2^24 for dim <= 256).
//
// A workgroup of 4 waves owns 256 query rows and one slice of the base
// columns.  Wave w owns rows [64w, 64w + 64) as 4 blocks of 16 whose int8
// operands stay in registers for the whole slice; the slice streams through
// LDS in tiles of 64 columns (two buffers: the next tile is fetched while the
// current one is multiplied), and each B fragment read from LDS feeds the
// 4 row blocks.  v_mfma_i32_16x16x32_i8: lane l supplies 8 bytes of row
// (l % 16) of A (resp. column (l % 16) of B) at k offset 8 * (l / 16); the
// result element i of lane l is C[4 * (l / 16) + i][l % 16].
//
// Selection.  A slice is visited in increasing column order, so a column can
// enter a row's best Kp only if its d2 is strictly below the Kp-th best d2
// seen so far (an equal d2 loses the tie to the smaller id already held).
// With t = |x'|^2 - thr per row, the test d2 < thr is 2 x'.y' - |y'|^2 > t:
// one shift-add and one compare per distance, and a wave ballot skips the
// append path when no lane passes.  Passing columns are appended to the
// row's buffer (global memory, cap entries of (d2 << 32 | column)); before a
// tile could overflow it, the owning wave sorts the buffer in LDS, keeps the
// best Kp and tightens thr.  A second kernel merges the slices of each row,
// drops the row's own column when asked, and writes the K best.
namespace i8 {

constexpr int kRowsWG = 256;
constexpr int kCols = 64;
constexpr int kMaxD = 256;
constexpr int32_t kInf = 1 << 24;       // above every d2 of the data
constexpr int32_t kPadNorm = 1 << 28;   // |y'|^2 of padding columns: never passes
constexpr int kRsrcWord3 = 0x00020000;  // buffer resource word 3 on gfx9-family parts (raw, 32-bit data)
constexpr int kWaitVmcnt0 = 0x0F70;     // s_waitcnt vmcnt(0), the other counters left alone
constexpr int kMaxMerged = 4096;        // slices x Kp entries merged per row
constexpr int kRing = 512;              // candidates a wave stages in LDS before writing them out

typedef int v4i __attribute__((ext_vector_type(4)));

struct Args {
    const int8_t *b8;
    const int32_t *bn;
    int64_t n;
    const int8_t *q8;
    const int32_t *qn;
    int64_t rows;
    int Kp;               // entries kept per (row, slice)
    int cap;              // buffer entries per (row, slice): power of two >= Kp + kCols
    int slices;
    int64_t slice_len;    // multiple of kCols
    uint64_t *buf;        // rows x slices x cap
    int32_t *cnt;         // rows x slices
    const int32_t *col_id;      // id reported for each column (NULL: its index)
    const int32_t *start_tile;  // per workgroup: the column tile its pass starts at (NULL: 0)
};

__host__ __device__ inline size_t stride_for(int ks) { return (size_t)ks * 32 + 8; }

// per wave: the candidate ring (kRing words and kRing (row, slot) tags), or
// the sort scratch of cap words, which is used only while the ring is empty
__host__ __device__ inline size_t wave_region(int cap)
{
    const size_t ring = (size_t)kRing * 12, sort = (size_t)cap * 8;
    return ring > sort ? ring : sort;
}

__host__ inline size_t tile_lds(int ks, int cap)
{
    return round_up(2 * kCols * stride_for(ks), 16) + 2 * kCols * 4 + 2 * kCols * 4 +
           3 * kRowsWG * 4 + 4 * wave_region(cap);
}

// One wave: sort the c entries of g through LDS scratch s, keep the best Kp
// in g (sorted); returns the kept count and sets thr to the Kp-th d2 (kInf
// while fewer are held).
__device__ inline int sort_keep(uint64_t *g, int c, int Kp, uint64_t *s, int32_t &thr)
{
    const int lane = __lane_id();
    int P = 64;
    while (P < c) P <<= 1;
    for (int t = lane; t < P; t += 64) s[t] = t < c ? g[t] : ~0ull;
    knn::wsync();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < P / 2; t += 64) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t x = s[lo], y = s[hi];
                if (up ? (y < x) : (x < y)) {
                    s[lo] = y;
                    s[hi] = x;
                }
            }
            knn::wsync();
        }
    }
    const int keep = c < Kp ? c : Kp;
    for (int t = lane; t < keep; t += 64) g[t] = s[t];
    thr = keep == Kp ? (int32_t)(s[Kp - 1] >> 32) : kInf;
    knn::wsync();
    return keep;
}

template <int KS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KS <= 4 ? 3 : 2))) tiles_kernel(Args a)
{
    constexpr int STRIDE = KS * 32 + 8;
    constexpr int CHUNKS = kCols * KS * 4;          // 8-byte chunks per tile
    constexpr int PER_T = (CHUNKS + 255) / 256;
    extern __shared__ __align__(16) unsigned char dyn[];
    int8_t *Bs = reinterpret_cast<int8_t *>(dyn);
    int32_t *Bn = reinterpret_cast<int32_t *>(dyn + (2 * kCols * STRIDE + 15) / 16 * 16);
    int32_t *Bid = Bn + 2 * kCols;          // the columns' reported ids
    int32_t *r_an = Bid + 2 * kCols;
    // per row: |q'|^2 - thr - 1, the bound the distance test compares with
    // (in LDS, read per column block, to leave registers to the operands)
    int32_t *r_tv = r_an + kRowsWG;
    int32_t *r_cnt = r_tv + kRowsWG;
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int lane = t & 63;
    unsigned char *region = reinterpret_cast<unsigned char *>(r_cnt + kRowsWG) + (size_t)w * wave_region(a.cap);
    uint64_t *scratch = reinterpret_cast<uint64_t *>(region);
    uint64_t *ring_w = scratch;                                        // (d2 << 32) | column
    uint32_t *ring_m = reinterpret_cast<uint32_t *>(region + (size_t)kRing * 8);   // (row << 16) | slot
    int ring_n = 0;          // candidates staged by this wave (uniform)
    const int64_t row0 = (int64_t)blockIdx.x * kRowsWG;
    const int slice = blockIdx.y;
    const int64_t c_begin = (int64_t)slice * a.slice_len;
    int64_t c_end = c_begin + a.slice_len;
    if (c_end > a.n) c_end = a.n;
    const int ntiles = c_end > c_begin ? (int)((c_end - c_begin + kCols - 1) / kCols) : 0;
    const int dim = KS * 32;
    // the pass visits the slice's tiles cyclically from start0 (the tiles of
    // the workgroup's own cluster first, when the rows are cluster-ordered)
    int start0 = a.start_tile ? a.start_tile[blockIdx.x] : 0;
    if (start0 < 0 || start0 >= ntiles) start0 = 0;
    auto tile_c0 = [&](int it) {
        int j = start0 + it;
        if (j >= ntiles) j -= ntiles;
        return c_begin + (int64_t)j * kCols;
    };

    {
        const int64_t g = row0 + t;
        r_an[t] = g < a.rows ? a.qn[g] : 0;
        r_tv[t] = g < a.rows ? a.qn[g] - kInf - 1 : 0x7fffffff;
        r_cnt[t] = 0;
    }
    // A operands: row block rb, k-step ks
    long long areg[4][KS];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t g = row0 + 64 * w + 16 * rb + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            areg[rb][ks] = g < a.rows ? *reinterpret_cast<const long long *>(
                                            a.q8 + g * dim + 32 * ks + 8 * (lane >> 4))
                                      : 0ll;
    }

    // Column tiles stream through a register stage and two LDS buffers: tile
    // it + 1 is requested while tile it is multiplied and written to LDS
    // after it.
    struct Stage {
        long long v[PER_T];
        int32_t n, id;
    };
    // Buffer loads through resources based at the tile's first column (in
    // scalar registers): each lane's offsets are the same for every tile, and
    // bytes past the end of the data read as zeros (those columns carry the
    // padding norm, so they never pass).
    int32_t boff[PER_T];
#pragma unroll
    for (int e = 0; e < PER_T; ++e) {
        const int ch = t + 256 * e;
        boff[e] = ch < CHUNKS ? (ch / (KS * 4)) * dim + 8 * (ch % (KS * 4)) : 0;
    }
    auto fetch = [&](int it, Stage &sg) {
        const int64_t c0 = tile_c0(it);
        const int64_t left = a.n - c0;
        const int cols = left < kCols ? (int)left : kCols;
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.b8 + c0 * dim), (short)0, cols * dim, kRsrcWord3);
#pragma unroll
        for (int e = 0; e < PER_T; ++e) {
            long long v = 0;
            if (CHUNKS % 256 == 0 || t + 256 * e < CHUNKS) {
                const auto u = __builtin_amdgcn_raw_buffer_load_b64(rb, boff[e], 0, 0);
                v = ((long long)u[1] << 32) | (uint32_t)u[0];
            }
            sg.v[e] = v;
        }
        const __amdgpu_buffer_rsrc_t rn = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.bn + c0), (short)0, cols * 4, kRsrcWord3);
        sg.n = t < kCols ? __builtin_amdgcn_raw_buffer_load_b32(rn, 4 * t, 0, 0) : 0;
        sg.id = (int32_t)(c0 + t);
        if (a.col_id) {
            const __amdgpu_buffer_rsrc_t ri = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.col_id + c0), (short)0, cols * 4, kRsrcWord3);
            sg.id = t < kCols ? __builtin_amdgcn_raw_buffer_load_b32(ri, 4 * t, 0, 0) : 0;
        }
    };
    auto store = [&](int it, int buf, const Stage &sg) {
        const int64_t c0 = tile_c0(it);
#pragma unroll
        for (int e = 0; e < PER_T; ++e) {
            const int ch = t + 256 * e;
            if (CHUNKS % 256 == 0 || ch < CHUNKS) {
                const int c = ch / (KS * 4), j = ch % (KS * 4);
                *reinterpret_cast<long long *>(Bs + (size_t)(buf * kCols + c) * STRIDE + 8 * j) =
                    sg.v[e];
            }
        }
        // negated, as the distance test adds it; columns past the slice get
        // the padding norm
        if (t < kCols) {
            Bn[buf * kCols + t] = c0 + t < c_end ? -sg.n : -kPadNorm;
            Bid[buf * kCols + t] = sg.id;
        }
    };

    // the staged candidates to their rows' buffer slots
    auto flush_ring = [&]() {
        const int m = ring_n < kRing ? ring_n : kRing;
        knn::wsync();
        for (int e = lane; e < m; e += 64) {
            const uint32_t tag = ring_m[e];
            a.buf[((row0 + (tag >> 16)) * a.slices + slice) * (int64_t)a.cap + (tag & 0xffffu)] =
                ring_w[e];
        }
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        knn::wsync();
        ring_n = 0;
    };

    Stage sg;
    if (ntiles > 0) {
        fetch(0, sg);
        store(0, 0, sg);
    }
    __syncthreads();
    for (int it = 0; it < ntiles; ++it) {
        const int cur = it & 1;
        // unrolled: a loop here makes the compiler wait for the tile loads in
        // flight before entering it
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int cl = 16 * cb + (lane & 15);
            long long bf[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                bf[ks] = *reinterpret_cast<const long long *>(
                    Bs + (size_t)(cur * kCols + cl) * STRIDE + 32 * ks + 8 * (lane >> 4));
            // the column's norm, negated in LDS so that 2 * dot - |x'|^2 is one
            // shift-and-add
            const int32_t nbc = Bn[cur * kCols + cl];
            // the four row blocks' products first (independent accumulators,
            // so the matrix core pipelines them), then the tests
            v4i acc[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                acc[rb] = v4i{0, 0, 0, 0};
                // pairs of 32-byte k-steps on the 64-deep CDNA4 instruction:
                // each lane's 16 bytes are its two 8-byte chunks, the same
                // (row or column, k) correspondence for both operands, so the
                // integer dot product is unchanged
#pragma unroll
                for (int ks = 0; ks + 1 < KS; ks += 2) {
                    const v4i av = {(int)areg[rb][ks], (int)(areg[rb][ks] >> 32),
                                    (int)areg[rb][ks + 1], (int)(areg[rb][ks + 1] >> 32)};
                    const v4i bv = {(int)bf[ks], (int)(bf[ks] >> 32), (int)bf[ks + 1],
                                    (int)(bf[ks + 1] >> 32)};
                    acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, acc[rb], 0, 0, 0);
                }
                if (KS & 1) {
                    // the odd last chunk with zeros beside it (the same
                    // instruction throughout: mixing the 32- and 64-deep forms
                    // on one accumulator gave wrong sums on the GPU)
                    const v4i av = {(int)areg[rb][KS - 1], (int)(areg[rb][KS - 1] >> 32), 0, 0};
                    const v4i bv = {(int)bf[KS - 1], (int)(bf[KS - 1] >> 32), 0, 0};
                    acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, acc[rb], 0, 0, 0);
                }
            }
            // 2 * dot - |x'|^2 > |q'|^2 - thr - 1  <=>  d2 <= thr: one shift-add
            // and one compare per distance, one ballot for the 16 of this
            // lane.  An equal d2 is let in (the sort orders ties by id), so
            // the columns may come in any order.
            bool p[4][4];
            bool any = false;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int4 tv = *reinterpret_cast<const int4 *>(r_tv + 64 * w + 16 * rb +
                                                                4 * (lane >> 4));
                p[rb][0] = (acc[rb][0] << 1) + nbc > tv.x;
                p[rb][1] = (acc[rb][1] << 1) + nbc > tv.y;
                p[rb][2] = (acc[rb][2] << 1) + nbc > tv.z;
                p[rb][3] = (acc[rb][3] << 1) + nbc > tv.w;
                any |= p[rb][0] | p[rb][1] | p[rb][2] | p[rb][3];
            }
            if (__builtin_amdgcn_ballot_w64(any)) {
                // a candidate takes its row's next buffer slot now and waits
                // in the wave's LDS ring; the ring goes out to the buffers in
                // one pass later (global stores here would keep the next
                // products waiting for them)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint64_t m = __builtin_amdgcn_ballot_w64(p[rb][i]);
                        if (!m) continue;
                        if (p[rb][i]) {
                            const int rl = 64 * w + 16 * rb + 4 * (lane >> 4) + i;
                            const int32_t d2 = r_an[rl] - nbc - 2 * acc[rb][i];
                            const int slot = atomicAdd(&r_cnt[rl], 1);
                            const uint64_t word = ((uint64_t)(uint32_t)d2 << 32) |
                                                  (uint32_t)Bid[cur * kCols + cl];
                            const int pos = ring_n + (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                            if (pos < kRing) {
                                ring_w[pos] = word;
                                ring_m[pos] = ((uint32_t)rl << 16) | (uint32_t)slot;
                            } else {
                                // ring full (the first tiles, where most pass)
                                a.buf[((row0 + rl) * a.slices + slice) * (int64_t)a.cap + slot] =
                                    word;
                            }
                        }
                        ring_n += __popcll(m);
                    }
                if (ring_n > kRing)
                    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);   // the direct stores, on this path only
            }
            // the next tile is requested after the first column block's
            // products: requested before them, the compiler waits for it there
            if (cb == 0 && it + 1 < ntiles) fetch(it + 1, sg);
        }
        // sort the rows whose buffers could not take another tile, after
        // writing the ring out; write it out anyway once it is half full
        knn::wsync();
        const int my = 64 * w + lane;
        uint64_t full = __builtin_amdgcn_ballot_w64(r_cnt[my] > a.cap - kCols);
        if (full || ring_n > kRing / 2) flush_ring();
        if (full) {
            while (full) {
                const int r = 64 * w + (int)__builtin_ctzll(full);
                full &= full - 1;
                int32_t thr;
                uint64_t *g = a.buf + ((row0 + r) * a.slices + slice) * (int64_t)a.cap;
                const int keep = sort_keep(g, r_cnt[r], a.Kp, scratch, thr);
                if (lane == 0) {
                    r_cnt[r] = keep;
                    r_tv[r] = r_an[r] - thr - 1;
                }
                knn::wsync();
            }
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);     // the sorts' stores, as above
        }
        if (it + 1 < ntiles) store(it + 1, cur ^ 1, sg);
        __syncthreads();
    }
    // final sort of every row of this wave; counts out
    flush_ring();
    for (int r = 64 * w; r < 64 * w + 64; ++r) {
        if (row0 + r >= a.rows) break;
        int c = r_cnt[r];
        if (c > 0) {
            int32_t thr;
            c = sort_keep(a.buf + ((row0 + r) * a.slices + slice) * (int64_t)a.cap, c, a.Kp,
                          scratch, thr);
        }
        if (lane == 0) a.cnt[(row0 + r) * a.slices + slice] = c;
    }
}

// One wave per row: the best Kp over the row's slices, the row's own column
// dropped when asked, the first K written (-1 / +inf padded).
__global__ void __launch_bounds__(64) select_kernel(const uint64_t *buf, const int32_t *cnt,
                                                    int64_t rows, int slices, int cap, int Kp,
                                                    int K, int exclude, const int32_t *self_col,
                                                    const int32_t *row_map, int32_t *out_ids,
                                                    float *out_f, double *out_d)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    uint64_t *s = reinterpret_cast<uint64_t *>(dyn);
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g >= rows) return;
    const uint64_t *list = buf + g * slices * (int64_t)cap;
    int total;
    if (slices == 1) {
        total = cnt[g];
    } else {
        // concatenate the sorted slice lists, then sort (bitonic) through LDS
        int c = 0;
        for (int sl = 0; sl < slices; ++sl) {
            const int m = cnt[g * slices + sl];
            for (int t = lane; t < m; t += 64) s[c + t] = list[(int64_t)sl * cap + t];
            c += m;
        }
        int P = 64;
        while (P < c) P <<= 1;
        for (int t = c + lane; t < P; t += 64) s[t] = ~0ull;
        knn::wsync();
        for (int size = 2; size <= P; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = lane; t < P / 2; t += 64) {
                    const int lo = 2 * t - (t & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t x = s[lo], y = s[hi];
                    if (up ? (y < x) : (x < y)) {
                        s[lo] = y;
                        s[hi] = x;
                    }
                }
                knn::wsync();
            }
        total = c < Kp ? c : Kp;
        list = s;
    }
    if (total > Kp) total = Kp;
    // position of the row's own column among the first `total` entries
    int self_at = total;
    if (exclude) {
        const uint32_t me = (uint32_t)(self_col ? self_col[g] : g);
        for (int t = lane; t < total; t += 64)
            if ((uint32_t)list[t] == me) self_at = t;
        for (int o = 32; o > 0; o >>= 1) {
            const int other = __shfl_xor(self_at, o);
            self_at = other < self_at ? other : self_at;
        }
    }
    const int have = total - (self_at < total ? 1 : 0);
    const int64_t go = row_map ? (int64_t)row_map[g] : g;     // the output row
    for (int o = lane; o < K; o += 64) {
        int32_t id = -1;
        double v = __longlong_as_double(0x7ff0000000000000ll);
        if (o < have) {
            const uint64_t e = list[o < self_at ? o : o + 1];
            id = (int32_t)(uint32_t)e;
            v = (double)(int32_t)(e >> 32);
        }
        out_ids[go * K + o] = id;
        if (out_f) out_f[go * K + o] = (float)v;
        if (out_d) out_d[go * K + o] = v;
    }
}

// ---- cluster order for all-pairs passes.  The rows are grouped by their
// nearest of kClusters sample rows (every (n / kClusters)-th row), and each
// workgroup visits the columns of its own group first: the best K of a row
// are then mostly seen early, its threshold is tight for the rest of the
// pass, and few columns reach the append path.  Only the visiting order
// changes; the selection is exact in any order.
constexpr int kClusters = 256;
constexpr int64_t kClusterMinN = 65536;   // below this the pass is short anyway

// the sample rows (int8) and their norms
__global__ void sample_rows_kernel(const int8_t *x8, const int32_t *xn, int64_t n, int dim,
                                   int C, int8_t *c8, int32_t *cn)
{
    const int c = blockIdx.x;
    const int64_t r = (int64_t)c * n / C;
    for (int j = threadIdx.x; j < dim; j += blockDim.x) c8[(size_t)c * dim + j] = x8[r * dim + j];
    if (threadIdx.x == 0) cn[c] = xn[r];
}

// nearest sample row of every row by (|c'|^2 - 2 x'.c', c), int8 dot products
// in 32-bit; the C sample rows sit in LDS
template <int W>
__global__ void __launch_bounds__(256) nearest_sample_kernel(const int8_t *x8, int64_t n,
                                                             const int8_t *c8, const int32_t *cn,
                                                             int C, int32_t *cid, int32_t *hist)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    int32_t *cs = reinterpret_cast<int32_t *>(dyn);                 // C x W packed int8
    int32_t *csn = cs + (size_t)C * W;
    for (int i = threadIdx.x; i < C * W; i += blockDim.x)
        cs[i] = reinterpret_cast<const int32_t *>(c8)[i];
    for (int i = threadIdx.x; i < C; i += blockDim.x) csn[i] = cn[i];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t xr[W];
#pragma unroll
    for (int k = 0; k < W; ++k) xr[k] = reinterpret_cast<const int32_t *>(x8 + r * (4 * W))[k];
    int best = 0;
    int32_t bv = 0x7fffffff;
    for (int c = 0; c < C; ++c) {
        const int32_t *cc = cs + (size_t)c * W;
        int32_t dot = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) dot = __builtin_amdgcn_sdot4(xr[k], cc[k], dot, false);
        const int32_t v = csn[c] - 2 * dot;
        if (v < bv) {
            bv = v;
            best = c;
        }
    }
    cid[r] = best;
    atomicAdd(&hist[best], 1);
}

// exclusive scan of the C group sizes (one thread; C is small): group starts
// in start[0..C], a running copy in fill[0..C), which may be hist itself
__global__ void group_starts_kernel(const int32_t *hist, int C, int32_t *start, int32_t *fill)
{
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int c = 0; c < C; ++c) {
            const int32_t h = hist[c];
            start[c] = acc;
            fill[c] = acc;
            acc += h;
        }
        start[C] = acc;
    }
}

// rows placed group by group (the order inside a group is whatever the
// atomics give; the results do not depend on it)
__global__ void place_rows_kernel(const int32_t *cid, int64_t n, int32_t *fill, int32_t *perm)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t pos = atomicAdd(&fill[cid[r]], 1);
    perm[pos] = (int32_t)r;
}

// the rows in group order: int8 rows and norms
__global__ void gather_rows8_kernel(const int8_t *x8, const int32_t *xn, const int32_t *perm,
                                    int64_t n, int dim, int8_t *y8, int32_t *yn)
{
    const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (p >= n) return;
    const int lane = threadIdx.x & 63;
    const int64_t r = perm[p];
    const int32_t *src = reinterpret_cast<const int32_t *>(x8 + r * dim);
    int32_t *dst = reinterpret_cast<int32_t *>(y8 + p * dim);
    for (int k = lane; k < dim / 4; k += 64) dst[k] = src[k];
    if (lane == 0) yn[p] = xn[r];
}

// each workgroup's first column tile: the start of the group of its first row
__global__ void start_tiles_kernel(const int32_t *cid, const int32_t *perm, const int32_t *start,
                                   int64_t n, int64_t blocks, int32_t *start_tile)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= blocks) return;
    const int64_t p = b * kRowsWG;
    start_tile[b] = p < n ? start[cid[perm[p]]] / kCols : 0;
}

struct Plan {
    int Kp, cap, slices;
    int64_t slice_len;
};

Plan plan(int64_t n, int64_t rows, int K)
{
    Plan p{};
    p.Kp = K + 1;          // room for the row's own column
    // a row's buffer holds its best Kp and at least one more tile; below 512
    // entries it also holds Kp more, so that a row is sorted at most once per
    // Kp new candidates
    p.cap = 64;
    while (p.cap < p.Kp + kCols || (p.cap < 512 && p.cap < 2 * p.Kp + kCols)) p.cap <<= 1;
    const int64_t blocks = (rows + kRowsWG - 1) / kRowsWG;
    int64_t s = (2048 + blocks - 1) / (blocks > 0 ? blocks : 1);
    const int64_t by_len = n / 4096 > 1 ? n / 4096 : 1;
    const int64_t by_merge = kMaxMerged / p.Kp > 1 ? kMaxMerged / p.Kp : 1;
    if (s > by_len) s = by_len;
    if (s > by_merge) s = by_merge;
    if (s < 1) s = 1;
    p.slice_len = ((n + s - 1) / s + kCols - 1) / kCols * kCols;
    p.slices = (int)((n + p.slice_len - 1) / p.slice_len);
    if (p.slices < 1) p.slices = 1;
    return p;
}

// all-pairs passes over enough rows run in cluster order
inline bool cluster_order(int64_t n, int64_t rows) { return rows == n && n >= kClusterMinN; }

size_t cluster_ws(int64_t n, int dim)
{
    const int64_t blocks = (n + kRowsWG - 1) / kRowsWG;
    return round_up((size_t)n * 4, 256) * 2 +                         // group of each row, order
           round_up((size_t)kClusters * dim, 256) + 3 * round_up((size_t)(kClusters + 1) * 4, 256) +
           round_up((size_t)blocks * 4, 256);
}

size_t workspace(int64_t n, int64_t rows, int dim, int K)
{
    const Plan p = plan(n, rows, K);
    size_t b = round_up((size_t)rows * p.slices * p.cap * 8, 256);
    b += round_up((size_t)rows * p.slices * 4, 256);
    b += round_up((size_t)n * dim, 256) + round_up((size_t)n * 4, 256);
    b += round_up((size_t)rows * dim, 256) + round_up((size_t)rows * 4, 256);
    if (cluster_order(n, rows)) b += cluster_ws(n, dim);
    return b + 256;
}

template <int KS>
ann_status launch_tiles(const Args &a, hipStream_t st)
{
    const size_t lds = tile_lds(KS, a.cap);
    ANN_HIP(hipFuncSetAttribute((const void *)tiles_kernel<KS>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    dim3 grid((unsigned)((a.rows + kRowsWG - 1) / kRowsWG), (unsigned)a.slices);
    hipLaunchKernelGGL(tiles_kernel<KS>, grid, dim3(256), lds, st, a);
    ANN_LAUNCHED();
    return ANN_OK;
}

}  // namespace i8

}  // namespace

size_t knn_cap(int K)
{
    size_t c = 2;
    while (c < (size_t)(K + F_BN)) c <<= 1;
    return c;
}

size_t knn_workspace(int64_t n, int64_t rows, int dim, int K)
{
    const size_t f64 = round_up((size_t)rows * knn_cap(K) * sizeof(Ent), 256) + 256;
    const size_t i8b = i8::workspace(n, rows, dim, K);
    return (f64 > i8b ? f64 : i8b) + 256;
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
    if (rows == 0) return ANN_OK;
    unsigned char *p = static_cast<unsigned char *>(ws);
    int *flag = reinterpret_cast<int *>(p);
    p += 256;
    bool use_int = false;
    if (force_engine != 2 && dim % 32 == 0 && dim <= i8::kMaxD) {
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
    if (use_int) {
        const i8::Plan pl = i8::plan(n, rows, K);
        i8::Args a{};
        a.buf = reinterpret_cast<uint64_t *>(p);
        p += round_up((size_t)rows * pl.slices * pl.cap * 8, 256);
        a.cnt = reinterpret_cast<int32_t *>(p);
        p += round_up((size_t)rows * pl.slices * 4, 256);
        int8_t *b8 = reinterpret_cast<int8_t *>(p);
        p += round_up((size_t)n * dim, 256);
        int32_t *bn = reinterpret_cast<int32_t *>(p);
        p += round_up((size_t)n * 4, 256);
        int8_t *q8 = reinterpret_cast<int8_t *>(p);
        p += round_up((size_t)rows * dim, 256);
        int32_t *qn = reinterpret_cast<int32_t *>(p);
        p += round_up((size_t)rows * 4, 256);
        const int32_t *row_map = nullptr;
        a.col_id = nullptr;
        a.start_tile = nullptr;
        if (queries == base && self_col == nullptr && i8::cluster_order(n, rows) &&
            n <= 0x7FFFFFFF) {
            // all pairs: rows and columns in the order of their nearest sample
            // row, ids reported through the permutation
            const int C = i8::kClusters;
            const int64_t blocks = (n + i8::kRowsWG - 1) / i8::kRowsWG;
            int32_t *cid = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)n * 4, 256);
            int32_t *perm = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)n * 4, 256);
            int8_t *c8 = reinterpret_cast<int8_t *>(p);
            p += round_up((size_t)C * dim, 256);
            int32_t *cn = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)(C + 1) * 4, 256);
            int32_t *hist = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)(C + 1) * 4, 256);
            int32_t *gstart = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)(C + 1) * 4, 256);
            int32_t *start_tile = reinterpret_cast<int32_t *>(p);
            p += round_up((size_t)blocks * 4, 256);
            hipLaunchKernelGGL(to_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st,
                               base, n, dim, q8, qn);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(i8::sample_rows_kernel, dim3(C), dim3(64), 0, st, q8, qn, n, dim, C,
                               c8, cn);
            ANN_LAUNCHED();
            ANN_HIP(hipMemsetAsync(hist, 0, (size_t)(C + 1) * 4, st));
            const size_t slds = (size_t)C * dim + (size_t)C * 4;
            const dim3 rg((unsigned)((n + 255) / 256));
            switch (dim / 32) {
#define ANN_NEAREST(W)                                                                              \
    case W / 8:                                                                                     \
        ANN_HIP(hipFuncSetAttribute((const void *)i8::nearest_sample_kernel<W>,                    \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)slds));       \
        hipLaunchKernelGGL(i8::nearest_sample_kernel<W>, rg, dim3(256), slds, st, q8, n, c8, cn,   \
                           C, cid, hist);                                                          \
        break;
                ANN_NEAREST(8) ANN_NEAREST(16) ANN_NEAREST(24) ANN_NEAREST(32)
                ANN_NEAREST(40) ANN_NEAREST(48) ANN_NEAREST(56) ANN_NEAREST(64)
#undef ANN_NEAREST
            default: return fail(ANN_ENOTSUP, "int8 engine: dim %d", dim);
            }
            ANN_LAUNCHED();
            // the group sizes become the running fill positions
            hipLaunchKernelGGL(i8::group_starts_kernel, dim3(1), dim3(64), 0, st, hist, C, gstart,
                               hist);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(i8::place_rows_kernel, rg, dim3(256), 0, st, cid, n, hist, perm);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(i8::gather_rows8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0,
                               st, q8, qn, perm, n, dim, b8, bn);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(i8::start_tiles_kernel, dim3((unsigned)((blocks + 255) / 256)),
                               dim3(256), 0, st, cid, perm, gstart, n, blocks, start_tile);
            ANN_LAUNCHED();
            a.b8 = b8;
            a.bn = bn;
            a.q8 = b8;
            a.qn = bn;
            a.col_id = perm;
            a.start_tile = start_tile;
            row_map = perm;
            self_col = perm;
        } else {
            hipLaunchKernelGGL(to_int8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st,
                               base, n, dim, b8, bn);
            ANN_LAUNCHED();
            hipLaunchKernelGGL(to_int8_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st,
                               queries, rows, dim, q8, qn);
            ANN_LAUNCHED();
            a.b8 = b8;
            a.bn = bn;
            a.q8 = q8;
            a.qn = qn;
        }
        a.n = n;
        a.rows = rows;
        a.Kp = pl.Kp;
        a.cap = pl.cap;
        a.slices = pl.slices;
        a.slice_len = pl.slice_len;
        ann_status s = ANN_OK;
        switch (dim / 32) {
        case 1: s = i8::launch_tiles<1>(a, st); break;
        case 2: s = i8::launch_tiles<2>(a, st); break;
        case 3: s = i8::launch_tiles<3>(a, st); break;
        case 4: s = i8::launch_tiles<4>(a, st); break;
        case 5: s = i8::launch_tiles<5>(a, st); break;
        case 6: s = i8::launch_tiles<6>(a, st); break;
        case 7: s = i8::launch_tiles<7>(a, st); break;
        default: s = i8::launch_tiles<8>(a, st); break;
        }
        if (s != ANN_OK) return s;
        const size_t lds = pl.slices > 1 ? (size_t)i8::kMaxMerged * 8 : 0;
        if (lds)
            ANN_HIP(hipFuncSetAttribute((const void *)i8::select_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(i8::select_kernel, dim3((unsigned)rows), dim3(64), lds, st, a.buf, a.cnt,
                           rows, pl.slices, pl.cap, pl.Kp, K, exclude_self ? 1 : 0, self_col,
                           row_map, out_ids, out_f, out_d);
        ANN_LAUNCHED();
    } else {
        KnnArgs a{};
        a.base = base;
        a.n = n;
        a.dim = dim;
        a.queries = queries;
        a.rows = rows;
        a.K = K;
        a.exclude_self = exclude_self ? 1 : 0;
        a.self_col = self_col;
        a.buf = reinterpret_cast<Ent *>(p);
        a.out_ids = out_ids;
        a.out_f = out_f;
        a.out_d = out_d;
        a.cap = (int)knn_cap(K);
        const int blocks = (int)((rows + knn::kRows - 1) / knn::kRows);
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
