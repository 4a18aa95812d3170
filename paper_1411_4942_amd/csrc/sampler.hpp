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
#include "ladder_wave.hpp"
#include "rowhash.hpp"

namespace pm {

// The adjacency tests a sample still needs after its picks: three row
// windows [lo, hi) with the key to look for, each the row of the pair's
// smaller id (after the relabel the shorter or equal row), except the
// 3-path sampler's y under the row hash (below).  3-path: x = [u'~v],
// y = [u~v'], z = [u'~v']; centered: the same three, z first.
struct SampleTests {
    uint32_t lo[3], hi[3], key[3];
};

constexpr uint32_t kUndecided = 0xFFu;

__device__ __forceinline__ void test_window(SampleTests &t, int i, uint32_t a, uint32_t alo, uint32_t ad, uint32_t b,
                                            uint32_t blo, uint32_t bd)
{
    const bool lo_a = a < b;
    t.lo[i] = lo_a ? alo : blo;
    t.hi[i] = t.lo[i] + (lo_a ? ad : bd);
    t.key[i] = lo_a ? b : a;
}

// Algorithms 1 and 3 from the picked slot s on: the neighbour picks from the
// offset o in [0, w_s) inside the slot's weight w_s (read by the centered
// sampler only), and the adjacency tests that classify the sample as in
// Algorithms 2 and 4.  Returns PM_TALLY_TRI when the picks coincide (the
// triangle outcome), else kUndecided with the tests filled.  Every record
// carries its column's row bounds, so each test knows its row without
// another load.  With ROW_U_FOR_Y (the row hash, where a test costs one line
// whatever the row's length) the 3-path sampler's y = [u~v'] probes row u
// itself: samples in draw order run through row u's slots one after another,
// so that row's hash lines are the ones most likely cached.
template <bool CENTERED, bool ROW_U_FOR_Y = false>
__device__ __forceinline__ uint32_t sample_picks(const SamplerView &g, uint32_t s, uint64_t o, uint64_t ws,
                                                 SampleTests &t)
{
    const SlotRec e = g.rec[s];
    const uint32_t u = e.row, v = e.col, ov = e.coff, dv = e.cdeg;
    const uint32_t ou = (uint32_t)g.off[u], du = (uint32_t)g.off[u + 1] - ou;
    const uint32_t pos_v = s - ou;  // position of v in row u

    SlotRec pu, pv;  // the picked slots: u' = pu.col, v' = pv.col
    if (!CENTERED) {
        // o in [0, (d_u-1)(d_v-1)): u' is the a-th of N(u)\{v} (v's own
        // position stands for the row's last entry), v' the b-th of N(v)\{u}
        uint64_t a, b;
        divmod_small(o, dv - 1, a, b);
        pu = g.rec[ou + ((uint32_t)a == pos_v ? du - 1 : (uint32_t)a)];
        pv = g.rec[ov + (uint32_t)b];
        if (pv.col == u) pv = g.rec[ov + dv - 1];
    } else {
        // o in [0, L_uv L_vu): u' among the L_uv neighbours of u after v, v'
        // among the L_vu neighbours of v after u (row suffixes)
        const uint32_t luv = du - 1 - pos_v;
        uint64_t lvu, rem, a, b;
        divmod_small(ws, luv, lvu, rem);
        divmod_small(o, (uint32_t)lvu, a, b);
        pu = g.rec[s + 1 + (uint32_t)a];
        pv = g.rec[ov + (dv - (uint32_t)lvu) + (uint32_t)b];
    }
    const uint32_t up = pu.col, vp = pv.col;
    if (up == vp) return PM_TALLY_TRI;
    // centered: v < u' and u < v' by construction, so x and y search the
    // rows of v and u
    test_window(t, 0, up, pu.coff, pu.cdeg, v, ov, dv);
    if (!CENTERED && ROW_U_FOR_Y) {
        t.lo[1] = ou;
        t.hi[1] = ou + du;
        t.key[1] = vp;
    } else {
        test_window(t, 1, u, ou, du, vp, pv.coff, pv.cdeg);
    }
    test_window(t, 2, up, pu.coff, pu.cdeg, vp, pv.coff, pv.cdeg);
    return kUndecided;
}

// 3-path classification (Algorithm 2) from x = [u'~v], y = [u~v'],
// z = [u'~v']: 3 edges: 3-path; 4: 4-cycle with the closing edge z, else
// tailed triangle; 5: chordal-4-cycle; 6: 4-clique.
__device__ __forceinline__ uint32_t classify_path(uint32_t x, uint32_t y, uint32_t z)
{
    const uint32_t edges = x + y + z;
    return edges == 0 ? 2u : edges == 1 ? (z ? 4u : 3u) : edges == 2 ? 5u : 6u;
}

// One adjacency test of a sample in this lane: key in the row window
// [lo, hi)?  SEARCH = PM_SEARCH_HASH probes the row hash, PM_SEARCH_LANE
// walks the ladder index; both give the same answer.
template <int SEARCH>
__device__ __forceinline__ uint32_t row_contains(const SamplerView &g, const SampleTests &t, int i)
{
    if (SEARCH == PM_SEARCH_HASH) return rowhash_contains(g.hash, t.lo[i], t.hi[i] - t.lo[i], t.key[i]) ? 1u : 0u;
    return ladder_contains(g.ladder, t.lo[i], t.hi[i], t.key[i]) ? 1u : 0u;
}

// Tally index of the sample at slot s (per-lane searches).  Centered
// (Algorithm 4): centered iff u'~v' (Definition 4.1); then the chords u'~v
// and u~v' give 4-cycle, chordal-4-cycle or 4-clique.
template <bool CENTERED, int SEARCH = PM_SEARCH_HASH>
__device__ __forceinline__ uint32_t sample_decode(const SamplerView &g, uint32_t s, uint64_t o, uint64_t ws)
{
    SampleTests t;
    const uint32_t pre = sample_picks<CENTERED, SEARCH == PM_SEARCH_HASH>(g, s, o, ws, t);
    if (pre != kUndecided) return pre;
    if (!CENTERED) {
        const uint32_t x = row_contains<SEARCH>(g, t, 0);
        const uint32_t y = row_contains<SEARCH>(g, t, 1);
        const uint32_t z = row_contains<SEARCH>(g, t, 2);
        return classify_path(x, y, z);
    } else {
        if (!row_contains<SEARCH>(g, t, 2)) return PM_TALLY_OPEN;
        const uint32_t x = row_contains<SEARCH>(g, t, 0);
        const uint32_t y = row_contains<SEARCH>(g, t, 1);
        return 4u + x + y;
    }
}

// global inclusive prefix of the sampler's weights at slot i
__device__ __forceinline__ uint64_t prefix_at(const SamplerView &g, uint32_t i)
{
    return g.P[i] + g.Pseg[i >> kPrefixSegShift];
}

// The edge draw of sample `id` (R > 0; positions below 2^32): r exact
// uniform in [0, R), its slot s = min{s : P[s] > r} from the guide table and
// a short binary search, the offset o = r - P[s-1] inside the slot's weight,
// and (centered only) that weight w_s.
template <bool CENTERED>
__device__ __forceinline__ uint32_t sample_slot(const SamplerView &g, uint64_t seed, uint64_t id, uint64_t &o,
                                                uint64_t &ws)
{
    const uint64_t r = draw_bounded(seed, CENTERED ? 1u : 0u, id, g.R);

    // window from the guide table.  Inside one prefix segment the search
    // compares the stored (segment) prefixes with r less the segment's
    // offset: one offset load instead of one per probe (a window nearly
    // always lies in one segment).
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
    o = r - below;
    ws = CENTERED ? g.P[s] - p_prev : 0ull;
    return s;
}

// Tally index of sample `id` (R > 0), per-lane searches.
template <bool CENTERED, int SEARCH = PM_SEARCH_HASH>
__device__ __forceinline__ uint32_t sample_class(const SamplerView &g, uint64_t seed, uint64_t id)
{
    uint64_t o, ws;
    const uint32_t s = sample_slot<CENTERED>(g, seed, id, o, ws);
    return sample_decode<CENTERED, SEARCH>(g, s, o, ws);
}

// Tally index of the sample in this lane (`active`) with the adjacency tests
// done by the wave together (ladder_contains_wave): every lane of the wave
// must call it, lanes without a sample pass active = false (the result is
// then meaningless).
template <bool CENTERED>
__device__ __forceinline__ uint32_t sample_class_wave(const SamplerView &g, uint64_t seed, uint64_t id, bool active)
{
    SampleTests t;
    uint32_t cls = kUndecided;
    if (active) {
        uint64_t o, ws;
        const uint32_t s = sample_slot<CENTERED>(g, seed, id, o, ws);
        cls = sample_picks<CENTERED>(g, s, o, ws, t);
    }
    const bool need = active && cls == kUndecided;
    if (!CENTERED) {
        const uint32_t x = ladder_contains_wave(g.ladder, need, t.lo[0], t.hi[0], t.key[0]) ? 1u : 0u;
        const uint32_t y = ladder_contains_wave(g.ladder, need, t.lo[1], t.hi[1], t.key[1]) ? 1u : 0u;
        const uint32_t z = ladder_contains_wave(g.ladder, need, t.lo[2], t.hi[2], t.key[2]) ? 1u : 0u;
        if (need) cls = classify_path(x, y, z);
    } else {
        const bool z = ladder_contains_wave(g.ladder, need, t.lo[2], t.hi[2], t.key[2]);
        const bool chords = need && z;
        const uint32_t x = ladder_contains_wave(g.ladder, chords, t.lo[0], t.hi[0], t.key[0]) ? 1u : 0u;
        const uint32_t y = ladder_contains_wave(g.ladder, chords, t.lo[1], t.hi[1], t.key[1]) ? 1u : 0u;
        if (need) cls = z ? 4u + x + y : (uint32_t)PM_TALLY_OPEN;
    }
    return cls;
}

// Draw-ordered sampling (pm_count, pm_sample_async, pm_count_alias): for at
// least draw_order_min() samples of one sampler, ids are sorted in chunks of
// kSortedChunk by the top kDrawKeyBits bits of their first draw before they
// run.  Measured on MI355X the sort pays from about 2M samples, for graphs
// from 7e6 to 2.4e8 slots alike (its fixed cost dominates below).
constexpr int kDrawKeyBits = 24;
constexpr uint64_t kSortedMinDefault = 1ull << 21;
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
