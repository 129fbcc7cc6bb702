// Wavefront-level building blocks of the best-first beam search
// (Algorithm 1 read as a bounded, sorted candidate pool).
//
// One wavefront (64 lanes) owns one query at a time.  Its state lives in a
// private slice of LDS:
//   pool   two ping-pong arrays of at most pool_cap entries (key, id), kept
//          sorted by (key, id); bit 31 of id marks "expanded"
//   stage  64 entries for the candidates of the current hop
//   vis    the visited filter: an exact bitset when the id range fits, else
//          an open-addressing table of ids that may forget an id when a probe
//          run is full but never reports an unseen id as seen
// Keys are order-preserving integer images of the FP32 (or FP64) distance,
// so comparisons are integer compares and ties fall to the smaller id.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ann {
namespace beam {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr int kMaxProbe = 32;

enum Metric { L2 = 0, NEG_IP = 1 };

template <bool F64> struct Key;
template <> struct Key<false> {
    using K = uint32_t;
    using D = float;
    static constexpr K kMax = 0xFFFFFFFFu;
    __device__ static inline K of(float f)
    {
        uint32_t u = __float_as_uint(f);
        return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    __device__ static inline float value(K k)
    {
        uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
        return __uint_as_float(u);
    }
};
template <> struct Key<true> {
    using K = uint64_t;
    using D = double;
    static constexpr K kMax = 0xFFFFFFFFFFFFFFFFull;
    __device__ static inline K of(double f)
    {
        uint64_t u = (uint64_t)__double_as_longlong(f);
        return (u >> 63) ? ~u : (u | (1ull << 63));
    }
    __device__ static inline float value(K k)
    {
        uint64_t u = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
        return (float)__longlong_as_double((long long)u);
    }
};

// (ka, ia) < (kb, ib) with the expanded bit ignored
template <typename K>
__device__ inline bool key_less(K ka, uint32_t ia, K kb, uint32_t ib)
{
    return ka < kb || (ka == kb && (ia & kIdMask) < (ib & kIdMask));
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline int lane_id() { return __lane_id(); }

// first index j in [0, cnt) with !(a[j] < key)
template <typename K>
__device__ inline int lower_bound(const K *ak, const uint32_t *ai, int cnt, K k, uint32_t id)
{
    int lo = 0, hi = cnt;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (key_less(ak[mid], ai[mid], k, id))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// ascending bitonic sort of one (key, id) per lane across the wavefront
template <typename K>
__device__ inline void wave_sort(K &k, uint32_t &id)
{
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            K ok = __shfl_xor(k, stride);
            uint32_t oi = __shfl_xor(id, stride);
            bool up = (lane & size) == 0;
            bool lower = (lane & stride) == 0;
            bool mine_less = key_less(k, id, ok, oi);
            bool keep = (lower == up) ? mine_less : !mine_less;
            if (!keep) {
                k = ok;
                id = oi;
            }
        }
    }
}

// ---------------------------------------------------------------- visited
struct Visited {
    uint32_t *t;
    int log2cap;
    bool bitset;   // exact bitset over [0, n)
    int words;     // slots to clear

    __device__ inline void clear() const
    {
        for (int i = lane_id(); i < words; i += 64) t[i] = bitset ? 0u : kEmpty;
        wave_sync();
    }

    // true if id was not seen before (and records it when there is room);
    // `lost` is set when the id could not be recorded.
    __device__ inline bool insert(uint32_t id, bool &lost) const
    {
        if (bitset) {
            uint32_t bit = 1u << (id & 31u);
            uint32_t old = atomicOr(&t[id >> 5], bit);
            return (old & bit) == 0;
        }
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = (id * 2654435761u) >> (32 - log2cap);
        for (int p = 0; p < kMaxProbe; ++p) {
            uint32_t slot = (h + (uint32_t)p) & mask;
            uint32_t old = atomicCAS(&t[slot], kEmpty, id);
            if (old == kEmpty || old == id) return old == kEmpty;
        }
        lost = true;
        return true;
    }
};

}  // namespace beam
}  // namespace ann
