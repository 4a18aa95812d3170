// Device-resident prepared graph (the pm_graph handle) and the view the
// sampling kernels take.
#pragma once

#include <vector>

#include "common.hpp"
#include "ladder.hpp"

namespace pm {

// What the samplers read about one slot s = (u, v) of the relabelled CSR, in
// one 16-byte load: its column v with v's row offset and degree, and its own
// row u.  A neighbour pick reads the record of the picked slot, so the picked
// vertex arrives with the bounds of its row (no separate offset gathers).
struct SlotRec {
    uint32_t col;   // v
    uint32_t coff;  // off[v]
    uint32_t cdeg;  // d_v
    uint32_t row;   // u
};
static_assert(sizeof(SlotRec) == 16, "slot record is 16 bytes");

}  // namespace pm

// Relabelled graph: vertex ids are positions in the degree order of Section 4
// (degree, then input id), so "u before v" is integer u < v and every row is
// sorted in that order.  Slot s is position s of the CSR; rec[s] is its
// sampler record.
struct pm_graph {
    int device = 0;
    int64_t n = 0;
    int64_t slots = 0;            // 2m
    uint32_t *off = nullptr;      // [n+1] (every slot index is below 2^32)
    uint32_t *col = nullptr;      // [slots]
    pm::SlotRec *rec = nullptr;   // [slots] column, its row offset and degree, row
    uint32_t *hash = nullptr;     // [2 slots + pad] row hash of the adjacency tests (rowhash.hpp)
    uint32_t *deg = nullptr;      // [n]
    int32_t *rank = nullptr;      // [n] input id -> relabelled id
    uint64_t *p_tau = nullptr;    // [slots] inclusive prefix of tau inside each kPrefixSeg-slot segment
    uint64_t *p_lam = nullptr;    // [slots] the same for lambda
    uint64_t *seg_tau = nullptr;  // [nseg + 1] tau before each segment; [nseg] = 2W
    uint64_t *seg_lam = nullptr;  // [nseg + 1] the same for lambda; [nseg] = 2 Lambda
    uint32_t *ladder = nullptr;   // levels 1..ladder_top of the row search index
    int ladder_top = 0;
    uint64_t ladder_off[8] = {0};  // start of level l inside `ladder`
    uint32_t *guide_tau = nullptr;  // [nb_tau + 1]
    uint32_t *guide_lam = nullptr;  // [nb_lam + 1]
    uint32_t shift_tau = 0, shift_lam = 0;
    uint64_t nb_tau = 0, nb_lam = 0;
    uint64_t R_tau = 0;  // 2W
    uint64_t R_lam = 0;  // 2 Lambda
    void *alias_tau = nullptr;  // [slots] alias-draw tables (pm::AliasEntry), built on request
    void *alias_lam = nullptr;
    uint64_t N1 = 0;
    int64_t dmax = 0;
    int64_t isolated = 0;
    uint64_t bytes = 0;
};

namespace pm {

// One bucket of an alias-draw table (32 bytes, so a draw reads one line):
// the bucket keeps K of its own slot's mass (capacity R) and holds R - K of
// slot `alias`; both slots' weights ride along for the position draw.
struct AliasEntry {
    uint64_t K;
    uint64_t w_self;
    uint64_t w_alias;
    uint32_t alias;
    uint32_t pad;
};
static_assert(sizeof(AliasEntry) == 32, "alias entry is 32 bytes");

// Prefix sums are stored per segment of kPrefixSeg slots (one wave of the
// weights pass): P[s] is the inclusive sum from the segment's first slot, and
// the global prefix is P[s] + seg[s >> kPrefixSegShift].
constexpr int kPrefixSegShift = 10;
constexpr int64_t kPrefixSeg = 1ll << kPrefixSegShift;

inline int64_t prefix_segments(int64_t slots) { return (slots + kPrefixSeg - 1) / kPrefixSeg; }

// Everything one sampler needs about one graph.
struct SamplerView {
    const uint32_t *off;
    const uint32_t *col;
    Ladder ladder;
    const SlotRec *rec;      // per-slot records
    const uint32_t *hash;    // row hash (rowhash.hpp)
    const uint64_t *P;       // inclusive prefix of the sampler's weights, per segment
    const uint64_t *Pseg;    // prefix before each segment
    const uint32_t *guide;   // guide[j] = first slot with P > j << shift
    uint64_t R;              // total weight (0: sampler skipped)
    uint32_t shift;
};

inline SamplerView view_of(const pm_graph *g, bool centered)
{
    SamplerView v;
    v.off = g->off;
    v.col = g->col;
    v.ladder.top = g->ladder_top;
    v.ladder.lvl[0] = g->col;
    for (int l = 1; l < kLadderMax; ++l) v.ladder.lvl[l] = l <= g->ladder_top ? g->ladder + g->ladder_off[l] : nullptr;
    v.rec = g->rec;
    v.hash = g->hash;
    v.P = centered ? g->p_lam : g->p_tau;
    v.Pseg = centered ? g->seg_lam : g->seg_tau;
    v.guide = centered ? g->guide_lam : g->guide_tau;
    v.R = centered ? g->R_lam : g->R_tau;
    v.shift = centered ? g->shift_lam : g->shift_tau;
    return v;
}

// device memory through the stream-ordered allocator
pm_status dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
// frees every non-null block of ps with one stream-ordered release point
void dev_free_batch(void *const *ps, size_t count, hipStream_t s);

// Scoped temporaries: every block still held is freed (stream-ordered) when
// the owner goes out of scope; keep() hands a block over to its new owner.
struct Temps {
    hipStream_t s;
    std::vector<void *> ptrs;
    explicit Temps(hipStream_t st) : s(st) {}
    ~Temps() { dev_free_batch(ptrs.data(), ptrs.size(), s); }
    template <typename T>
    pm_status get(T **p, size_t count)
    {
        void *q = nullptr;
        PM_TRY(dev_alloc(&q, count * sizeof(T), s));
        ptrs.push_back(q);
        *p = (T *)q;
        return PM_OK;
    }
    void release(void *p)
    {
        for (auto &q : ptrs)
            if (q == p) {
                dev_free(q, s);
                q = nullptr;
            }
    }
    void keep(void *p)
    {
        for (auto &q : ptrs)
            if (q == p) q = nullptr;
    }
};

}  // namespace pm
