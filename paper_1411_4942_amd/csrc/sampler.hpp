// One sample of Algorithm 1 classified as in Algorithm 2, or of Algorithm 3
// classified as in Algorithm 4, on a prepared graph (shared by the
// single-graph, batched and alias-draw kernels).
//   r      exact uniform in [0, R) from Philox keyed by (seed, id)
//   slot   first s with P[s] > r: guide table, then a short binary search
//   picks  o = r - P[s-1] split in mixed radix into the two neighbour picks
//   tests  the adjacency tests in the shorter row (after the relabel the
//          smaller id has the shorter or equal row), through the ladder
#pragma once

#include "graph.hpp"

namespace pm {

// Bounds of the row to search for the pair (known, other): the row of the
// smaller id; the offsets are loaded only when that row is not already in
// registers.
struct RowSearch {
    uint32_t lo, hi, key;
};

__device__ __forceinline__ RowSearch row_search(const uint32_t *__restrict__ off, uint32_t known, uint32_t klo,
                                                uint32_t khi, uint32_t other)
{
    if (known < other) return RowSearch{klo, khi, other};
    return RowSearch{(uint32_t)off[other], (uint32_t)off[other + 1], known};
}

__device__ __forceinline__ RowSearch row_search2(const uint32_t *__restrict__ off, uint32_t a, uint32_t b)
{
    const uint32_t x = a < b ? a : b;
    return RowSearch{(uint32_t)off[x], (uint32_t)off[x + 1], a < b ? b : a};
}

// Tally index of the sample at slot s with offset o in [0, w_s) inside the
// slot's weight w_s (Algorithms 1 and 3 from the picked edge on, classified
// as in Algorithms 2 and 4).  w_s is read by the centered sampler only.
template <bool CENTERED>
__device__ __forceinline__ uint32_t sample_decode(const SamplerView &g, uint32_t s, uint64_t o, uint64_t ws)
{
    const uint64_t e = g.edge[s];
    const uint32_t u = (uint32_t)e, v = (uint32_t)(e >> 32);
    const uint32_t ou = (uint32_t)g.off[u], du = (uint32_t)g.off[u + 1] - ou;
    const uint32_t ov = (uint32_t)g.off[v], dv = (uint32_t)g.off[v + 1] - ov;
    const uint32_t pos_v = s - ou;  // position of v in row u

    uint32_t up, vp;
    if (!CENTERED) {
        // o in [0, (d_u-1)(d_v-1)): u' is the a-th of N(u)\{v} (v's own
        // position stands for the row's last entry), v' the b-th of N(v)\{u}
        uint64_t a, b;
        divmod_small(o, dv - 1, a, b);
        up = g.col[ou + ((uint32_t)a == pos_v ? du - 1 : (uint32_t)a)];
        vp = g.col[ov + (uint32_t)b];
        if (vp == u) vp = g.col[ov + dv - 1];
    } else {
        // o in [0, L_uv L_vu): u' among the L_uv neighbours of u after v, v'
        // among the L_vu neighbours of v after u (row suffixes)
        const uint32_t luv = du - 1 - pos_v;
        uint64_t lvu, rem, a, b;
        divmod_small(ws, luv, lvu, rem);
        divmod_small(o, (uint32_t)lvu, a, b);
        up = g.col[s + 1 + (uint32_t)a];
        vp = g.col[ov + (dv - (uint32_t)lvu) + (uint32_t)b];
    }
    if (up == vp) return PM_TALLY_TRI;

    if (!CENTERED) {
        // x = [u'~v], y = [u~v'], z = [u'~v']
        const RowSearch sx = row_search(g.off, v, ov, ov + dv, up);
        const RowSearch sy = row_search(g.off, u, ou, ou + du, vp);
        const RowSearch sz = row_search2(g.off, up, vp);
        const uint32_t x = ladder_contains(g.ladder, sx.lo, sx.hi, sx.key);
        const uint32_t y = ladder_contains(g.ladder, sy.lo, sy.hi, sy.key);
        const uint32_t z = ladder_contains(g.ladder, sz.lo, sz.hi, sz.key);
        const uint32_t edges = x + y + z;
        // 3 edges: 3-path; 4: 4-cycle with the closing edge, else tailed
        // triangle; 5: chordal-4-cycle; 6: 4-clique
        return edges == 0 ? 2u : edges == 1 ? (z ? 4u : 3u) : edges == 2 ? 5u : 6u;
    } else {
        // centered iff u'~v' (Definition 4.1); then the chords u'~v and u~v',
        // searched in the rows of v and u (v < u' and u < v')
        const RowSearch sz = row_search2(g.off, up, vp);
        if (!ladder_contains(g.ladder, sz.lo, sz.hi, sz.key)) return PM_TALLY_OPEN;
        const uint32_t x = ladder_contains(g.ladder, ov, ov + dv, up);
        const uint32_t y = ladder_contains(g.ladder, ou, ou + du, vp);
        return 4u + x + y;
    }
}

// global inclusive prefix of the sampler's weights at slot i
__device__ __forceinline__ uint64_t prefix_at(const SamplerView &g, uint32_t i)
{
    return g.P[i] + g.Pseg[i >> kPrefixSegShift];
}

// Tally index of sample `id` (R > 0; positions below 2^32): r exact uniform
// in [0, R), its slot from the guide table and a short binary search.
template <bool CENTERED>
__device__ __forceinline__ uint32_t sample_class(const SamplerView &g, uint64_t seed, uint64_t id)
{
    const uint64_t r = draw_bounded(seed, CENTERED ? 1u : 0u, id, g.R);

    // edge draw: s = min{s : P[s] > r}, window from the guide table.  Inside
    // one prefix segment the search compares the stored (segment) prefixes
    // with r less the segment's offset: one offset load instead of one per
    // probe (a window nearly always lies in one segment).
    const uint64_t j = r >> g.shift;
    uint32_t lo = g.guide[j], hi = g.guide[j + 1];
    const uint32_t sg = lo >> kPrefixSegShift;
    const uint64_t off_sg = g.Pseg[sg];
    if (hi == lo || ((hi - 1) >> kPrefixSegShift) == sg) {
        const uint64_t rl = r - off_sg;  // slots before lo have prefix <= r, so rl >= 0
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (g.P[mid] > rl)
                hi = mid;
            else
                lo = mid + 1;
        }
    } else {
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (prefix_at(g, mid) > r)
                hi = mid;
            else
                lo = mid + 1;
        }
    }
    const uint32_t s = lo;
    // the global prefix just before a segment is that segment's offset
    const bool first = (s & (kPrefixSeg - 1)) == 0;
    const uint64_t p_prev = first ? 0ull : g.P[s - 1];
    const uint64_t below = ((s >> kPrefixSegShift) == sg ? off_sg : g.Pseg[s >> kPrefixSegShift]) + p_prev;
    return sample_decode<CENTERED>(g, s, r - below, CENTERED ? g.P[s] - p_prev : 0ull);
}

// Draw-ordered sampling (pm_count, pm_sample_async, pm_count_alias): for at
// least draw_order_min() samples of one sampler, ids are sorted in chunks of
// kSortedChunk by the top kDrawKeyBits bits of their first draw before they
// run.  Measured on MI355X the sort pays from about 4M samples, for graphs
// from 1e6 to 2.4e8 slots alike (its fixed cost dominates below).
constexpr int kDrawKeyBits = 24;
constexpr uint64_t kSortedMinDefault = 6ull << 20;
constexpr uint64_t kSortedChunk = 1ull << 24;  // samples per sort (bounds the temporaries)

bool draw_order_enabled();
uint64_t draw_order_min();

__device__ __forceinline__ void tally_add(uint32_t (&cnt)[PM_NUM_TALLIES], uint32_t cls)
{
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] += (cls == (uint32_t)c);
}

// per-lane counters -> one atomic per wave per class
__device__ __forceinline__ void tally_flush(const uint32_t (&cnt)[PM_NUM_TALLIES], unsigned long long *tally)
{
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) {
        const uint32_t t = wave_sum_u32(cnt[c]);
        if (lane_id() == 0 && t) atomicAdd(&tally[c], (unsigned long long)t);
    }
}

}  // namespace pm
