// The per-wavefront search engine used by the search, entry-selection and
// label kernels.  See search.hip for the algorithm and its invariants.
#pragma once

#include "beam.h"

namespace ann {

struct SearchArgs {
    const float *base;
    int64_t n;
    int dim;
    const int32_t *graph;
    int R;
    const float *queries;
    int nq;
    const int32_t *entry;
    int medoid;
    const int32_t *k;
    const int32_t *L;
    int k_max;
    int32_t *out_ids;
    float *out_dist;
    int32_t *stats;
    int32_t *trace;
    int trace_cap;
    int pool_cap;
    int visited_log2;
    beam::FilterShape filter;
    uint32_t *counter;
    const int32_t *order;   // NULL, or the order in which the queries are taken
    size_t wave_lds;
};

struct SearchResult {
    int ndc_exec;
    int dups;
    int hops;
    bool lost;
};

// Pools merged from registers (FP32 keys, at most 512 entries) are written
// back in place, so they need one buffer; the general merge reads one
// buffer and writes the other.
inline __host__ __device__ bool pool_in_place(int pool_cap, bool f64)
{
    return !f64 && pool_cap <= 512;
}

// LDS bytes one wavefront needs: the query vector, one or two pool buffers of
// (key, id), the staging row of 64 (key, id) and the visited filter's words.
inline size_t wave_lds_bytes(int pool_cap, const beam::FilterShape &f, bool f64, int dim)
{
    size_t ks = f64 ? 8 : 4;
    size_t bufs = pool_in_place(pool_cap, f64) ? 1 : 2;
    size_t b = ((size_t)dim * 4 + 15) / 16 * 16 + bufs * (size_t)pool_cap * ks + 64 * ks +
               bufs * (size_t)pool_cap * 4 + 64 * 4 + 64 + (size_t)f.words * 4;
    return (b + 15) / 16 * 16;
}

template <int G, int CPL, bool F64, int FILT>
struct Searcher {
    using KT = beam::Key<F64>;
    using K = typename KT::K;
    using D = typename KT::D;
    static constexpr int VPB = 64 / G;
    static constexpr int U0 = 16 / VPB;
    static constexpr int U1 = 16 / CPL;
    static constexpr int U = (U0 < U1 ? U0 : U1) < 1 ? 1 : (U0 < U1 ? U0 : U1);

    K *pk0, *pk1;
    uint32_t *pi0, *pi1;
    K *sk;
    uint32_t *si;
    beam::Visited<FILT> vis;
    int pool_cap;
    int64_t n;
    const float4 *base4;
    int chunks;
    const int32_t *graph;
    int R;
    float4 *ql;   // the query vector, in LDS
    int cur;
    int cnt;

    __device__ void setup(unsigned char *lds, int pcap, int vlog2, const beam::FilterShape &fs,
                          int64_t n_, const float *base, int dim, const int32_t *graph_, int R_)
    {
        const size_t ks = sizeof(K);
        const bool one = pool_in_place(pcap, F64);
        unsigned char *p = lds;
        ql = reinterpret_cast<float4 *>(p);
        p += ((size_t)dim * 4 + 15) / 16 * 16;
        pk0 = reinterpret_cast<K *>(p);
        p += pcap * ks;
        pk1 = pk0;
        if (!one) {
            pk1 = reinterpret_cast<K *>(p);
            p += pcap * ks;
        }
        sk = reinterpret_cast<K *>(p);
        p += 64 * ks;
        pi0 = reinterpret_cast<uint32_t *>(p);
        p += pcap * 4;
        pi1 = pi0;
        if (!one) {
            pi1 = reinterpret_cast<uint32_t *>(p);
            p += pcap * 4;
        }
        si = reinterpret_cast<uint32_t *>(p);
        p += 64 * 4;
        p += 64;
        vis.t = reinterpret_cast<uint32_t *>(p);
        vis.words = fs.words;
        vis.log2cap = vlog2;
        vis.tag_bits = fs.tag_bits;
        vis.hmask = fs.hmask;
        pool_cap = pcap;
        n = n_;
        base4 = reinterpret_cast<const float4 *>(base);
        chunks = dim / 4;
        graph = graph_;
        R = R_;
    }

    __device__ void load_query(const float *qp)
    {
        const float4 *q4 = reinterpret_cast<const float4 *>(qp);
        for (int ch = beam::lane_id(); ch < chunks; ch += 64) ql[ch] = q4[ch];
        beam::wave_sync();
    }

    __device__ inline K *keys(int c) const { return c ? pk1 : pk0; }
    __device__ inline uint32_t *ids(int c) const { return c ? pi1 : pi0; }

    __device__ static inline D partial(const float4 &x, const float4 &y)
    {
        D a = (D)x.x - (D)y.x, b = (D)x.y - (D)y.y, c = (D)x.z - (D)y.z, d = (D)x.w - (D)y.w;
        return a * a + b * b + c * c + d * d;
    }

    // keys of the m candidates si[0..m) into sk[0..m); with W waves sharing
    // the work, wave w takes every W-th batch of VPB * U candidates
    template <int W = 1>
    __device__ void distances(int m, int w = 0)
    {
        if (chunks == G * CPL)
            distances_impl<W, true>(m, w);
        else
            distances_impl<W, false>(m, w);
    }

    // FULL: every lane's CPL chunks lie inside the vector (dim == 4 * G * CPL),
    // so loads and sums need no per-lane bounds test.  A batch slot row whose
    // candidates all lie past m is skipped (a uniform test); inside a partly
    // valid row, lanes past m load the row's first candidate again and drop
    // the result.
    template <int W, bool FULL>
    __device__ void distances_impl(int m, int w)
    {
        const int lane = beam::lane_id();
        const int gi = lane / G, gl = lane % G;
        for (int b0 = w * VPB * U; b0 < m; b0 += W * VPB * U) {
            float4 xv[U][CPL];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cb = b0 + u * VPB;
                if (cb < m) {
                    const int c = cb + gi;
                    const uint32_t id = si[c < m ? c : cb];
                    const float4 *row = base4 + (size_t)id * chunks;
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int ch = gl + G * t;
                        xv[u][t] = (FULL || ch < chunks) ? row[ch] : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int cb = b0 + u * VPB;
                if (cb < m) {
                    D acc = 0;
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const int ch = gl + G * t;
                        if (FULL || ch < chunks) acc += partial(xv[u][t], ql[ch]);
                    }
                    acc = beam::group_sum<G>(acc);
                    const int c = cb + gi;
                    if (gl == 0 && c < m) sk[c] = KT::of(acc);
                }
            }
        }
        beam::wave_sync();
    }

    // first two pool positions at or after `from` whose entries are not
    // expanded (-1 when missing): one ballot usually yields both
    __device__ void next_two_unexpanded(int from, int &first, int &second) const
    {
        const int lane = beam::lane_id();
        const uint32_t *ai = ids(cur);
        first = -1;
        second = -1;
        for (int b = from; b < cnt; b += 64) {
            const int j = b + lane;
            const bool un = j < cnt && !(ai[j] & beam::kExpanded);
            uint64_t bal = __ballot(un);
            if (!bal) continue;
            if (first < 0) {
                first = b + __ffsll((unsigned long long)bal) - 1;
                bal &= bal - 1;
                if (!bal) continue;
            }
            second = b + __ffsll((unsigned long long)bal) - 1;
            return;
        }
    }

    // Merge for FP32 keys and pools of at most 64 * CM entries.  Lane l reads
    // pool entries l, l + 64, ... as 64-bit words (key << 32 | id, expanded
    // bit masked and kept aside for the write-back).  One pass over the
    // new keys gives each new key its insertion point (the count of smaller
    // pool words: one compare mask per word) and its rank among the new
    // keys, and each pool entry the count of new keys above it.  A new key
    // equal to the pool entry at its insertion point is a rediscovered node:
    // it is dropped and taken back out of the counts.  Then new key l goes
    // to place pos + rank and pool entry j to j + (new keys below it), all
    // at once, back into the same buffer (every read of the pool is done
    // before the first write).
    template <int CM>
    __device__ __forceinline__ void merge_words(int m, int Lq, int &cursor, uint32_t &pf_id,
                                                int &pf_nb, K nkey, uint32_t nid, SearchResult &r)
    {
        const int lane = beam::lane_id();
        const K *ak = keys(cur);
        const uint32_t *ai = ids(cur);
        // entries past cnt are read too (they lie inside the wave's LDS:
        // each pool array is followed by at least 64 entries of another) and
        // replaced by ~0; lane + 64 c < cnt is tested as lane < cnt - 64 c
        uint64_t P[CM];
        uint32_t ex = 0;   // expanded bits, bit c for word c
#pragma unroll
        for (int c = 0; c < CM; ++c) {
            const uint32_t id = ai[lane + 64 * c];
            const uint64_t w = ((uint64_t)ak[lane + 64 * c] << 32) | (id & beam::kIdMask);
            ex |= (id >> 31) << c;
            P[c] = lane < cnt - 64 * c ? w : ~0ull;
        }
        bool valid = lane < m;
        K kk = KT::kMax;
        uint32_t ii = beam::kEmpty;
        uint64_t S = ~0ull;
        if (valid) {
            kk = sk[lane];
            ii = si[lane];
            S = ((uint64_t)kk << 32) | ii;
        }
        // a full pool takes only keys below its last entry (a word below
        // ~0: ids are below 2^31)
        if (cnt == Lq) {
            const uint64_t last = ((uint64_t)ak[cnt - 1] << 32) | (ai[cnt - 1] & beam::kIdMask);
            valid = valid && S < last;
        }
        const uint64_t vmask = __ballot(valid);
        if (!vmask) return;
        int ltc[CM];
#pragma unroll
        for (int c = 0; c < CM; ++c) ltc[c] = 0;
        int rank = 0, pos = 0;
        for (uint64_t mm = vmask; mm; mm &= mm - 1) {
            const int t = __ffsll((unsigned long long)mm) - 1;
            const uint64_t s = beam::readlane(S, t);
            int below = 0;
#pragma unroll
            for (int c = 0; c < CM; ++c) {
                const bool lt = P[c] < s;
                below += __popcll(__ballot(lt));
                ltc[c] += lt ? 1 : 0;
            }
            pos = lane == t ? below : pos;
            rank += s < S ? 1 : 0;
        }
        // rediscovered nodes (a forgetful filter's repeats): equal to the
        // pool entry at their insertion point
        bool dup = false;
        if (valid) {
            const int pj = pos < cnt ? pos : 0;
            dup = pos < cnt && ak[pj] == kk && (ai[pj] & beam::kIdMask) == ii;
        }
        const uint64_t dmask = __ballot(dup);
        const int nv = __popcll(vmask);
        int mv = nv;
        if (dmask) {
            r.dups += __popcll(dmask);
            mv -= __popcll(dmask);
            if (mv == 0) return;
            for (uint64_t mm = dmask; mm; mm &= mm - 1) {
                const int t = __ffsll((unsigned long long)mm) - 1;
                const uint64_t s = beam::readlane(S, t);
                const int pt = __builtin_amdgcn_readlane(pos, t);
#pragma unroll
                for (int c = 0; c < CM; ++c) ltc[c] += (lane >= pt - 64 * c) ? 1 : 0;
                rank -= s < S ? 1 : 0;
            }
            valid = valid && !dup;
        }
        // the smallest new key: expanded next if it beats the old pool's
        // next unexpanded entry
        const int l0 = __ffsll((unsigned long long)__ballot(valid && rank == 0)) - 1;
        const K k0 = beam::readlane(kk, l0);
        const uint32_t i0 = beam::readlane(ii, l0);
        const int f0 = beam::readlane(pos, l0);
        if (beam::key_less(k0, i0, nkey, nid)) {
            pf_id = i0;
            pf_nb = lane < R ? graph[(size_t)i0 * R + lane] : -1;
        }
        // the pool's reads are all done: the merged pool goes to the same
        // buffer (keys(cur ^ 1) is keys(cur) for pools merged in place)
        beam::wave_sync();
        K *bk = keys(cur ^ 1);
        uint32_t *bi = ids(cur ^ 1);
        const int outn = __builtin_amdgcn_readfirstlane((cnt + mv < Lq) ? cnt + mv : Lq);
        const int fnew = pos + rank;
        if (valid && fnew < Lq) {
            bk[fnew] = kk;
            bi[fnew] = ii;
        }
#pragma unroll
        for (int c = 0; c < CM; ++c) {
            const int o = lane + (64 * c + nv) - ltc[c];
            if (lane < cnt - 64 * c && o < outn) {
                bk[o] = (K)(P[c] >> 32);
                bi[o] = (uint32_t)P[c] | (((ex >> c) & 1u) << 31);
            }
        }
        // the cursor's entry moves up by the new keys below it
        const int oc = cursor + __popcll(__ballot(valid && pos <= cursor));
        cursor = __builtin_amdgcn_readfirstlane(f0 < oc ? f0 : oc);
        cnt = outn;
        cur ^= 1;
        beam::wave_sync();
    }

    // Merges the m new keys (sk/si) into the pool.  Updates the cursor and,
    // when the best new key will be expanded next, the prefetched row.
    __device__ __forceinline__ void merge(int m, int Lq, int &cursor, uint32_t &pf_id, int &pf_nb,
                                          K nkey, uint32_t nid, SearchResult &r)
    {
        if constexpr (!F64) {
            // the pools that pool_in_place gives one buffer
            if (pool_cap <= 64) return merge_words<1>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 128) return merge_words<2>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 192) return merge_words<3>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 256) return merge_words<4>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 320) return merge_words<5>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 384) return merge_words<6>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 448) return merge_words<7>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            if (pool_cap <= 512) return merge_words<8>(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
        }
        merge_search(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
    }

    // The general merge (FP64 keys, or pools past 512 entries): insertion
    // points by binary search, ranks by a scalar loop over the new keys,
    // occupancy bits for the old entries' places.
    __device__ __forceinline__ void merge_search(int m, int Lq, int &cursor, uint32_t &pf_id,
                                                 int &pf_nb, K nkey, uint32_t nid, SearchResult &r)
    {
        const int lane = beam::lane_id();
        // ---- merge the new keys into the pool.  A new key's place is its
        // insertion point in the old pool plus its rank among the new keys
        // (a scalar loop over the new keys, readlane).  The new keys' places
        // are marked in a bit mask; every unmarked place takes the old entry
        // whose index is the place minus the marked places before it.  The
        // insertion points, stored by rank, give the cursor's new place.
        K *ak = keys(cur);
        uint32_t *ai = ids(cur);
        K kk = KT::kMax;
        uint32_t ii = beam::kEmpty;
        bool valid = lane < m;
        if (valid) {
            kk = sk[lane];
            ii = si[lane];
        }
        if (valid && cnt == Lq && !beam::key_less(kk, ii, ak[cnt - 1], ai[cnt - 1])) valid = false;
        int pos = 0;
        bool dup = false;
        if (valid) {
            pos = beam::lower_bound_uniform(ak, ai, cnt, kk, ii);
            if (pos < cnt && ak[pos] == kk && (ai[pos] & beam::kIdMask) == ii) dup = true;
        }
        valid = valid && !dup;
        r.dups += __popcll(__ballot(dup));
        const uint64_t vmask = __ballot(valid);
        const int mv = __popcll(vmask);
        if (mv == 0) return;
        int rank = 0;
        for (uint64_t mm = vmask; mm; mm &= mm - 1) {
            const int t = __ffsll((unsigned long long)mm) - 1;
            // new ids carry no expanded bit
            if (beam::pair_less(beam::readlane(kk, t), beam::readlane(ii, t), kk, ii)) ++rank;
        }
        // the smallest new key: expanded next if it beats the old pool's
        // next unexpanded entry
        const int l0 = __ffsll((unsigned long long)__ballot(valid && rank == 0)) - 1;
        const K k0 = beam::readlane(kk, l0);
        const uint32_t i0 = beam::readlane(ii, l0);
        const int f0 = beam::readlane(pos, l0);
        if (beam::key_less(k0, i0, nkey, nid)) {
            pf_id = i0;
            pf_nb = lane < R ? graph[(size_t)i0 * R + lane] : -1;
        }
        K *bk = keys(cur ^ 1);
        uint32_t *bi = ids(cur ^ 1);
        const int fnew = pos + rank;
        const bool placed = valid && fnew < Lq;
        if (placed) {
            bk[fnew] = kk;
            bi[fnew] = ii;
        }
        // insertion points by rank (the staging ids are in registers now)
        int32_t *sp = reinterpret_cast<int32_t *>(si);
        if (valid) sp[rank] = pos;
        // occupancy bits of the new keys' places in the merged pool (the
        // staging keys are in registers too, so their LDS holds the bits)
        const int outn = __builtin_amdgcn_readfirstlane((cnt + mv < Lq) ? cnt + mv : Lq);
        const int nw = (outn + 63) >> 6;
        uint32_t *occ = reinterpret_cast<uint32_t *>(sk);
        if (lane < 2 * nw) occ[lane] = 0u;
        beam::wave_sync();
        if (placed) atomicOr(&occ[fnew >> 5], 1u << (fnew & 31));
        beam::wave_sync();
        // every other place o takes old entry o - (new keys placed before o):
        // a count of the bits below the lane in the place's 64-bit word
        int before = 0;
        for (int c = 0; c < nw; ++c) {
            const uint32_t lo = __builtin_amdgcn_readfirstlane(occ[2 * c]);
            const uint32_t hi = __builtin_amdgcn_readfirstlane(occ[2 * c + 1]);
            const int o = (c << 6) + lane;
            const uint32_t word = lane < 32 ? lo : hi;
            if (o < outn && !((word >> (lane & 31)) & 1u)) {
                const int j = o - before -
                              (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
                const K kv = ak[j];
                const uint32_t iv = ai[j];
                bk[o] = kv;
                bi[o] = iv;
            }
            before += __popc(lo) + __popc(hi);
        }
        const int oc = cursor + beam::count_at_most(sp, mv, cursor);
        // cursor and count are the same in every lane; say so, so that they
        // stay in scalar registers
        cursor = __builtin_amdgcn_readfirstlane(f0 < oc ? f0 : oc);
        cnt = outn;
        cur ^= 1;
        beam::wave_sync();
    }

    // Runs one query from `entry` with beam width Lq.  trace (nullable)
    // receives the expanded ids.
    //
    // Latency hiding: the node expanded after p is either the old pool's next
    // unexpanded entry or, when one beats it, the best new neighbour of p.
    // The first one's adjacency row is loaded while p's neighbours are
    // gathered; if a new neighbour wins, its row is loaded before the merge.
    // A prefetched row is used only when its id is the node actually
    // expanded, so the expansion order does not depend on the prediction.
    __device__ SearchResult run(uint32_t entry, int Lq, int32_t *trace, int trace_cap)
    {
        const int lane = beam::lane_id();
        SearchResult r{0, 0, 0, false};
        vis.clear();
        bool lost = false;
        if (lane == 0) {
            vis.insert(entry, lost);
            si[0] = entry;
        }
        beam::wave_sync();
        distances(1);
        cur = 0;
        if (lane == 0) {
            pk0[0] = sk[0];
            pi0[0] = entry;
        }
        cnt = 1;
        r.ndc_exec = 1;
        beam::wave_sync();
        int cursor = 0;
        uint32_t pf_id = beam::kEmpty;
        int pf_nb = -1;
        for (;;) {
            int ppos, npos;
            next_two_unexpanded(cursor, ppos, npos);
            if (ppos < 0) break;
            cursor = ppos;
            const uint32_t p = ids(cur)[ppos] & beam::kIdMask;
            int nb = -1;
            if (p == pf_id)
                nb = pf_nb;
            else if (lane < R)
                nb = graph[(size_t)p * R + lane];
            K nkey = KT::kMax;
            uint32_t nid = beam::kEmpty;
            if (npos >= 0) {
                nkey = keys(cur)[npos];
                nid = ids(cur)[npos] & beam::kIdMask;
            }
            beam::wave_sync();
            if (lane == 0) {
                ids(cur)[ppos] = p | beam::kExpanded;
                if (trace && r.hops < trace_cap) trace[r.hops] = (int32_t)p;
            }
            r.hops++;
            // visited filter, compaction in slot order
            bool fresh = false;
            if (nb >= 0 && (int64_t)nb < n) fresh = vis.insert((uint32_t)nb, lost);
            uint64_t fb = __ballot(fresh);
            const int m = __popcll(fb);
            if (fresh) si[__popcll(fb & ((1ull << lane) - 1ull))] = (uint32_t)nb;
            // the old pool's next unexpanded row, requested once this row is
            // through the filter: requested before, the wait for this row
            // would wait for it as well
            pf_id = nid;
            if (npos >= 0) pf_nb = lane < R ? graph[(size_t)nid * R + lane] : -1;
            beam::wave_sync();
            if (m == 0) continue;
            distances(m);
            r.ndc_exec += m;
            merge(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
        }
        r.lost = __ballot(lost) != 0;
        return r;
    }

    // The same search with W wavefronts of one workgroup per query.  Wave 0
    // picks the node to expand, runs the visited filter and the merge; all W
    // waves gather and reduce the new neighbours' distances (every W-th batch
    // each).  ctrl (LDS, shared by the workgroup) carries the hop's count of
    // new neighbours, -1 when the search is over.  Every wave of the group
    // must call this with the same arguments; the barriers are workgroup-wide.
    template <int W>
    __device__ SearchResult run_multi(uint32_t entry, int Lq, int32_t *trace, int trace_cap, int w,
                                      volatile int *ctrl)
    {
        const int lane = beam::lane_id();
        SearchResult r{0, 0, 0, false};
        bool lost = false;
        int cursor = 0;
        uint32_t pf_id = beam::kEmpty;
        int pf_nb = -1;
        K nkey = KT::kMax;
        uint32_t nid = beam::kEmpty;
        if (w == 0) {
            vis.clear();
            if (lane == 0) {
                vis.insert(entry, lost);
                si[0] = entry;
            }
            beam::wave_sync();
            distances(1);
            cur = 0;
            if (lane == 0) {
                pk0[0] = sk[0];
                pi0[0] = entry;
            }
            cnt = 1;
            r.ndc_exec = 1;
            beam::wave_sync();
        }
        for (;;) {
            if (w == 0) {
                int m = -1;
                int ppos, npos;
                next_two_unexpanded(cursor, ppos, npos);
                if (ppos >= 0) {
                    cursor = ppos;
                    const uint32_t p = ids(cur)[ppos] & beam::kIdMask;
                    int nb = -1;
                    if (p == pf_id)
                        nb = pf_nb;
                    else if (lane < R)
                        nb = graph[(size_t)p * R + lane];
                    nkey = KT::kMax;
                    nid = beam::kEmpty;
                    pf_id = beam::kEmpty;
                    if (npos >= 0) {
                        nkey = keys(cur)[npos];
                        nid = ids(cur)[npos] & beam::kIdMask;
                        pf_id = nid;
                        pf_nb = lane < R ? graph[(size_t)nid * R + lane] : -1;
                    }
                    beam::wave_sync();
                    if (lane == 0) {
                        ids(cur)[ppos] = p | beam::kExpanded;
                        if (trace && r.hops < trace_cap) trace[r.hops] = (int32_t)p;
                    }
                    r.hops++;
                    bool fresh = false;
                    if (nb >= 0 && (int64_t)nb < n) fresh = vis.insert((uint32_t)nb, lost);
                    const uint64_t fb = __ballot(fresh);
                    m = __popcll(fb);
                    if (fresh) si[__popcll(fb & ((1ull << lane) - 1ull))] = (uint32_t)nb;
                }
                if (lane == 0) ctrl[0] = m;
            }
            __syncthreads();
            const int m = ctrl[0];
            if (m < 0) break;
            if (m > 0) distances<W>(m, w);
            __syncthreads();
            if (w == 0 && m > 0) {
                r.ndc_exec += m;
                merge(m, Lq, cursor, pf_id, pf_nb, nkey, nid, r);
            }
        }
        r.lost = __ballot(lost) != 0;
        return r;
    }

    __device__ void write_topk(int kq, int k_max, int32_t *oid, float *odist)
    {
        const int lane = beam::lane_id();
        const K *ak = keys(cur);
        const uint32_t *ai = ids(cur);
        for (int t = lane; t < k_max; t += 64) {
            int32_t id = -1;
            float dv = __int_as_float(0x7f800000);
            if (t < kq && t < cnt) {
                id = (int32_t)(ai[t] & beam::kIdMask);
                dv = KT::value(ak[t]);
            }
            oid[t] = id;
            odist[t] = dv;
        }
    }
};

// the several-wavefronts-per-query kernels (search_mw.hip)
ann_status launch_search_mw(const SearchArgs &a, int waves_per_query, int blocks, hipStream_t st);

}  // namespace ann
