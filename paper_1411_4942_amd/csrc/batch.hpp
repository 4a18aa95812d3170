// Work tiles of the persistent sampling kernel, shared by the batched and the
// served paths.
#pragma once

#include "graph.hpp"

namespace pm {

struct BatchGraph {
    SamplerView v[2];  // 3-path, centered
};

// A tile is (graph, sampler, first sample id, count, seed); its tallies go
// to slot `slot` (8 counters per sampler, 16 per slot).
struct BatchTile {
    uint32_t graph;
    uint32_t tag;    // 0 3-path sampler, 1 centered sampler
    uint32_t count;  // samples
    uint32_t slot;   // tally slot
    uint64_t first;  // first sample id
    uint64_t seed;
};

constexpr uint32_t kTileLists = 8;  // one tile list per XCD of an MI355X

// With nlists = 0 every block takes tiles from one cursor over [0, ntiles).
// With nlists > 0 the table is cut into nlists lists, list x holding tiles
// [begin[x], begin[x+1]); block b starts on list b mod nlists (consecutive
// blocks go to consecutive XCDs, so each XCD works through its own graphs
// and keeps their lines in its own L2) and, once that list is exhausted,
// helps with the next ones.
struct BatchCtl {
    uint32_t ntiles;
    uint32_t cursor;
    uint32_t nlists;
    uint32_t begin[kTileLists + 1];
    uint32_t lcursor[kTileLists];
};

// Enqueue the persistent kernel: `blocks` blocks take tiles from ctl's
// cursors until every tile is done, adding into tallies[slot * 16 + tag * 8 + c].
pm_status launch_tiles(const BatchGraph *graphs, const BatchTile *tiles, BatchCtl *ctl, uint64_t *tallies,
                       unsigned blocks, hipStream_t s);

}  // namespace pm
