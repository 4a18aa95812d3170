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

struct BatchCtl {
    uint32_t ntiles;
    uint32_t cursor;
};

// Enqueue the persistent kernel: `blocks` blocks take tiles from ctl->cursor
// until ctl->ntiles are done, adding into tallies[slot * 16 + tag * 8 + c].
pm_status launch_tiles(const BatchGraph *graphs, const BatchTile *tiles, BatchCtl *ctl, uint64_t *tallies,
                       unsigned blocks, hipStream_t s);

}  // namespace pm
