// Wavefront-level building blocks of the best-first beam search
// (Algorithm 1 read as a bounded, sorted candidate pool).
//
// One wavefront (64 lanes) owns one query at a time.  Its state lives in a
// private slice of LDS:
//   pool   one array (merged in place) or two ping-pong arrays of at most
//          pool_cap entries (key, id), kept
//          sorted by (key, id); bit 31 of id marks "expanded"
//   stage  64 entries for the candidates of the current hop
//   vis    the visited filter: an exact bitset when the id range fits, else
//          a hash table (16-bit tags or 32-bit ids) that may forget an id but
//          never reports an unseen id as seen
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

// the same order for ids whose expanded bit is already clear: one 64-bit
// compare of (key, id) for 32-bit keys
__device__ inline bool pair_less(uint32_t ka, uint32_t ia, uint32_t kb, uint32_t ib)
{
    return (((uint64_t)ka << 32) | ia) < (((uint64_t)kb << 32) | ib);
}
__device__ inline bool pair_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib)
{
    return (ka < kb) | ((ka == kb) & (ia < ib));
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The lane's index, opaque to the optimiser: values derived from it (LDS and
// global addresses of per-lane rows) are then recomputed where they are used
// instead of being hoisted out of the hop loop and held in registers for the
// whole launch, which keeps the search kernel's register count down.
__device__ inline int lane_id()
{
    int l = __lane_id();
    asm volatile("" : "+v"(l));
    return l;
}

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

// The same count with a step count that depends on cnt only (uniform across
// the wavefront): steps of 2^t from the largest power of two <= cnt down to
// 1, each adding its step when the entry ending that step is below the key.
// Branch-free per lane (probes past cnt are clamped and ignored).
// cnt must hold the same value in every active lane: it is read from the
// first one, so that the step count lives in a scalar register and the loop
// needs no per-lane exec masking.  Every probe reads a clamped index and the
// tests combine without short-circuit, so the body has no branch.
template <typename K>
__device__ inline int lower_bound_uniform(const K *ak, const uint32_t *ai, int cnt, K k, uint32_t id)
{
    cnt = __builtin_amdgcn_readfirstlane(cnt);
    if (cnt <= 0) return 0;
    const uint32_t idm = id & kIdMask;
    int lo = 0;
    for (int step = 1 << (31 - __builtin_clz((unsigned)cnt)); step > 0; step >>= 1) {
        const int probe = lo + step - 1;
        const int j = probe < cnt ? probe : cnt - 1;
        const bool below = (probe < cnt) & pair_less(ak[j], ai[j] & kIdMask, k, idm);
        lo += below ? step : 0;
    }
    return lo;
}

// number of entries <= x in the non-decreasing a[0..cnt), by fixed steps;
// cnt as for lower_bound_uniform
__device__ inline int count_at_most(const int32_t *a, int cnt, int x)
{
    cnt = __builtin_amdgcn_readfirstlane(cnt);
    if (cnt <= 0) return 0;
    int lo = 0;
    for (int step = 1 << (31 - __builtin_clz((unsigned)cnt)); step > 0; step >>= 1) {
        const int probe = lo + step - 1;
        const bool in = (probe < cnt) & (a[probe < cnt ? probe : cnt - 1] <= x);
        lo += in ? step : 0;
    }
    return lo;
}

// value of v in lane t (t uniform across the wavefront)
__device__ inline uint32_t readlane(uint32_t v, int t)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, t);
}
__device__ inline int readlane(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ inline uint64_t readlane(uint64_t v, int t)
{
    return ((uint64_t)readlane((uint32_t)(v >> 32), t) << 32) | readlane((uint32_t)v, t);
}

// Sum over aligned groups of G lanes (G = 8 or 16); every lane of a group
// receives the group's sum.  FP32 uses DPP lane moves: swap neighbours, swap
// pairs, then mirror within 8 lanes (and within 16 for G = 16); FP64 uses
// xor shuffles.
template <int CTRL>
__device__ inline float dpp_move(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int G>
__device__ inline float group_sum(float v)
{
    static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
    v += dpp_move<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);     // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_move<0x141>(v);    // row_half_mirror
    if (G == 16) v += dpp_move<0x140>(v);   // row_mirror
    return v;
}

template <int G>
__device__ inline double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------- visited
//
// Three forms, chosen per launch:
//   kBitset  one bit per id in [0, n): exact.
//   kTag16   4-way set-associative table of 16-bit tags.  An odd-constant
//            multiply modulo 2^b (b = bits of n) is a bijection on [0, 2^b);
//            its top bits pick the set and the rest is the tag, so (set, tag)
//            names exactly one id and a tag match is never a false "seen".
//            A set keeps its four newest tags; a fifth pushes out the
//            oldest (the evicted id is forgotten).
//   kTag12   the same hashing with five 12-bit ways per 64-bit set (tags of
//            at most 11 bits, so the all-ones way is never a tag): 25 % more
//            slots than kTag16 in the same bytes.
//   kId32    open-addressing table of 32-bit ids with bounded linear probing;
//            an id that finds no free slot in the probe run is not recorded.
// Forgetting is safe for the results (see the search kernel's header) and is
// reported through `lost`.
enum FilterKind { kBitset = 1, kTag16 = 2, kId32 = 3, kTag12 = 4 };

constexpr uint32_t kHashMul = 0x9E3779B1u;
constexpr uint32_t kTagEmpty = 0xFFFFu;

// KIND is the filter form, fixed at compile time so that one kernel holds
// the code (and the registers) of one form only.
template <int KIND>
struct Visited {
    static_assert(KIND == kBitset || KIND == kTag16 || KIND == kId32 || KIND == kTag12,
                  "filter form");
    uint32_t *t;
    int words;          // 32-bit words to clear
    int log2cap;        // kId32: slots; kTag16: slots (4 per set); kTag12: 4 x sets
    int tag_bits;       // tag forms: b - log2(sets), <= 15 (kTag16) or <= 11 (kTag12)
    uint32_t hmask;     // tag forms: 2^b - 1

    __device__ inline void clear() const
    {
        const uint32_t v = KIND == kBitset ? 0u : kEmpty;
        for (int i = lane_id(); i < words; i += 64) t[i] = v;
        wave_sync();
    }

    // true if id was not seen before (and records it when it can); `lost` is
    // set when an id could not be recorded or another was evicted.
    __device__ inline bool insert(uint32_t id, bool &lost) const
    {
        if (KIND == kBitset) {
            uint32_t bit = 1u << (id & 31u);
            uint32_t old = atomicOr(&t[id >> 5], bit);
            return (old & bit) == 0;
        }
        if (KIND == kTag16) return insert_tag(id, lost);
        if (KIND == kTag12) return insert_tag12(id, lost);
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = (id * kHashMul) >> (32 - log2cap);
#pragma unroll 1
        for (int p = 0; p < kMaxProbe; ++p) {
            uint32_t slot = (h + (uint32_t)p) & mask;
            uint32_t old = atomicCAS(&t[slot], kEmpty, id);
            if (old == kEmpty || old == id) return old == kEmpty;
        }
        lost = true;
        return true;
    }

    // 16-bit halves are tested two at a time (SWAR): a half of x is zero
    // exactly when its bit 15 survives (x - 0x00010001) & ~x; a borrow into
    // the upper half only arises when the lower half is zero, which is
    // checked first.
    __device__ static inline uint32_t zero_halves(uint32_t x)
    {
        return (x - 0x00010001u) & ~x & 0x80008000u;
    }

    __device__ inline bool insert_tag(uint32_t id, bool &lost) const
    {
        const uint32_t h = (id * kHashMul) & hmask;
        const uint32_t set = h >> tag_bits;
        const uint32_t tag = h & ((1u << tag_bits) - 1u);
        const uint32_t rep = tag * 0x00010001u;
        // a set is one 64-bit word of four 16-bit ways, newest in the low
        // half: a new tag is shifted in and the oldest way falls out (first
        // in, first out), so no way has to be chosen
        unsigned long long *w = reinterpret_cast<unsigned long long *>(t) + set;
#pragma unroll 1
        for (int it = 0; it < 8; ++it) {
            const unsigned long long old = __atomic_load_n(w, __ATOMIC_RELAXED);
            const uint32_t w0 = (uint32_t)old, w1 = (uint32_t)(old >> 32);
            if (zero_halves(w0 ^ rep) | zero_halves(w1 ^ rep)) return false;
            const unsigned long long nw = (old << 16) | tag;
            if (atomicCAS(w, old, nw) == old) {
                if ((uint32_t)(old >> 48) != kTagEmpty) lost = true;
                return true;
            }
        }
        lost = true;
        return true;
    }

    // Five 12-bit ways in bits 0..59 of a 64-bit set word, newest lowest; a
    // way of x is zero exactly when (x - ones) & ~x keeps its top bit (the
    // same borrow argument as for the 16-bit halves, over five fields).  A
    // cleared set reads all ones: every way is 0xFFF, above any 11-bit tag.
    __device__ inline bool insert_tag12(uint32_t id, bool &lost) const
    {
        constexpr unsigned long long kOnes = 0x001001001001001ull;
        constexpr unsigned long long kTops = 0x800800800800800ull;
        constexpr unsigned long long kWays = 0x0FFFFFFFFFFFFFFFull;
        const uint32_t h = (id * kHashMul) & hmask;
        const uint32_t set = h >> tag_bits;
        const unsigned long long tag = h & ((1u << tag_bits) - 1u);
        const unsigned long long rep = tag * kOnes;
        unsigned long long *w = reinterpret_cast<unsigned long long *>(t) + set;
#pragma unroll 1
        for (int it = 0; it < 8; ++it) {
            const unsigned long long old = __atomic_load_n(w, __ATOMIC_RELAXED);
            const unsigned long long x = old ^ rep;
            if ((x - kOnes) & ~x & kTops) return false;
            const unsigned long long nw = ((old << 12) | tag) & kWays;
            if (atomicCAS(w, old, nw) == old) {
                if (((old >> 48) & 0xFFFu) != 0xFFFu) lost = true;
                return true;
            }
        }
        lost = true;
        return true;
    }
};

// Filter layout for a launch: kind, table words and tag width.  kind_req 0
// picks the bitset when it is no larger than the table, else kTag12 when the
// tag fits in 11 bits, else kTag16 when it fits in 15, else kId32.  Returns
// false for a form that cannot hold n (a bitset larger than the table, or
// tags wider than the form's ways allow).  Both tag forms use 2^log2cap / 4
// sets of 64 bits.
struct FilterShape {
    int kind, words, tag_bits;
    uint32_t hmask;
};

__host__ __device__ inline int bits_for(int64_t n)
{
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n) ++b;
    return b;
}

__host__ __device__ inline bool filter_shape(int kind_req, int log2cap, int64_t n, FilterShape &f)
{
    const int64_t bitset_words = (n + 31) / 32;
    const int sets_log2 = log2cap - 2;
    int b = bits_for(n);
    if (b < sets_log2) b = sets_log2;
    const int tbits = b - sets_log2;
    int kind = kind_req;
    if (kind == 0)
        kind = bitset_words <= ((int64_t)1 << log2cap) / 2
                   ? kBitset
                   : (tbits <= 11 ? kTag12 : (tbits <= 15 ? kTag16 : kId32));
    f.kind = kind;
    f.tag_bits = tbits;
    f.hmask = b >= 32 ? 0xFFFFFFFFu : (uint32_t)(((uint64_t)1 << b) - 1u);
    if (kind == kBitset) {
        f.words = (int)bitset_words;
        return bitset_words <= ((int64_t)1 << log2cap);
    }
    if (kind == kTag16 || kind == kTag12) {
        f.words = 1 << (log2cap - 1);
        return tbits <= (kind == kTag16 ? 15 : 11);
    }
    if (kind == kId32) {
        f.words = 1 << log2cap;
        return true;
    }
    return false;
}

}  // namespace beam
}  // namespace ann
