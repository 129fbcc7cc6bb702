// Exact k-nearest-neighbour selection shared by the kNN engines.
//
// A workgroup owns a block of 64 query rows and streams every base column
// past them.  Each row keeps a threshold key (its current K-th best) in LDS;
// a distance whose key (d2, id) beats the threshold is appended to the row's
// candidate buffer in global memory.  Rows are owned by wavefronts (16 rows
// per wave), so when a row's buffer is close to full its wave sorts it
// (bitonic, in LDS), keeps the K best and tightens the threshold without any
// block-wide synchronisation.  Every key that could be in the final top K is
// appended (it beats the threshold at that time, which is never tighter than
// the final K-th key), so the final sort yields the exact top K by (d2, id).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ann {
namespace knn {

struct Ent {
    uint64_t k;    // order-preserving image of the distance
    uint32_t id;
    uint32_t pad;
};

constexpr uint64_t kMaxK = 0xFFFFFFFFFFFFFFFFull;
constexpr int kRows = 64;        // rows per workgroup
constexpr int kRowsPerWave = 16;

__device__ inline bool less(const Ent &a, const Ent &b)
{
    return a.k < b.k || (a.k == b.k && a.id < b.id);
}

__device__ inline Ent ent_max()
{
    Ent e;
    e.k = kMaxK;
    e.id = 0xFFFFFFFFu;
    e.pad = 0;
    return e;
}

__device__ inline uint64_t key_of(double v)
{
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

__device__ inline double value_of(uint64_t k)
{
    uint64_t u = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
    return __longlong_as_double((long long)u);
}

__device__ inline void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wave-level: sort row r's buffer (cnt entries) and keep the best K.
// scratch: cap entries of LDS private to the calling wave.
__device__ inline void merge_row(Ent *gbuf, int cap, int K, Ent *scratch, Ent &thr, int &cnt)
{
    const int lane = __lane_id();
    const int c = cnt;
    int P = 1;
    while (P < c) P <<= 1;
    if (P < 2) P = 2;
    for (int t = lane; t < P; t += 64) scratch[t] = t < c ? gbuf[t] : ent_max();
    wsync();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < P / 2; t += 64) {
                int lo = 2 * t - (t & (stride - 1));
                int hi = lo + stride;
                bool up = (lo & size) == 0;
                Ent a = scratch[lo], b = scratch[hi];
                bool swap = up ? less(b, a) : less(a, b);
                if (swap) {
                    scratch[lo] = b;
                    scratch[hi] = a;
                }
            }
            wsync();
        }
    }
    const int keep = c < K ? c : K;
    for (int t = lane; t < keep; t += 64) gbuf[t] = scratch[t];
    thr = (keep == K) ? scratch[K - 1] : ent_max();
    cnt = keep;
    wsync();
    (void)cap;
}

}  // namespace knn
}  // namespace ann
