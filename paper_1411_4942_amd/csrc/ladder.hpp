// Row search index ("ladder") over the column array of a CSR graph.
//
// Level 0 is the column array itself; level l >= 1 holds col[i * 32^l] at
// index i, so an aligned 32-entry (128-byte) line of level l covers 32^(l+1)
// slots.  A membership search in a sorted row starts at the lowest level
// whose samples inside the row share one line and reads one whole line per
// level, instead of a binary search's log2(row length) scattered probes.
// Every level (and the column array) is padded to whole lines, so a line
// read never leaves its allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pm {

constexpr int kLadderMax = 7;  // 32^7 = 2^35 covers every slot count below 2^32

struct Ladder {
    const uint32_t *lvl[kLadderMax];
    int top;  // highest level; its single line covers every slot
};

// smallest top with 32^(top+1) >= slots
__host__ __device__ inline int ladder_top_for(int64_t slots)
{
    int top = 0;
    const uint64_t s = slots > 1 ? (uint64_t)slots : 1u;
    while (top + 1 < kLadderMax && (1ull << (5 * (top + 1))) < s) ++top;
    return top;
}

// entries of level l >= 1: ceil(slots / 32^l)
__host__ __device__ inline uint64_t ladder_count(int64_t slots, int l)
{
    return ((uint64_t)slots + (1ull << (5 * l)) - 1) >> (5 * l);
}

// Is `key` in the ascending slot range [lo, hi)?  At each level the count of
// samples <= key narrows the range to the 32^l slots after the last of them
// (or to the slots before the first); the line is read with eight 16-byte
// loads and compared in registers.
__host__ __device__ inline bool ladder_contains(const Ladder &L, uint32_t lo, uint32_t hi, uint32_t key)
{
    if (lo >= hi) return false;
    int l = 0;
    while (l < L.top) {  // lowest level whose samples inside [lo, hi) share one line
        const uint32_t sh = 5u * l;
        const uint64_t a = ((uint64_t)lo + (1ull << sh) - 1) >> sh, b = (uint64_t)(hi - 1) >> sh;
        if (a > b || (a >> 5) == (b >> 5)) break;
        ++l;
    }
    uint64_t a = lo, b = hi;  // slot window holding the last entry <= key
    for (;; --l) {
        const uint32_t sh = 5u * l;
        const uint64_t first = (a + (1ull << sh) - 1) >> sh, last = (b - 1) >> sh;
        if (first <= last) {
            const uint64_t cell = first >> 5;
            const uint4 *line = reinterpret_cast<const uint4 *>(L.lvl[l] + cell * 32);
            uint4 w[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) w[t] = line[t];
            const uint32_t j0 = (uint32_t)(first - cell * 32), j1 = (uint32_t)(last - cell * 32);
            uint32_t cnt = 0;
            bool eq = false;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t e[4] = {w[t].x, w[t].y, w[t].z, w[t].w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint32_t j = 4u * t + c;
                    const bool in = j >= j0 && j <= j1;
                    cnt += (in && e[c] <= key) ? 1u : 0u;
                    eq |= in && e[c] == key;
                }
            }
            if (eq) return true;
            if (l == 0) return false;
            if (cnt == 0) {
                const uint64_t p = first << sh;
                b = b < p ? b : p;
            } else {
                const uint64_t i = first + cnt - 1;
                a = i << sh;
                const uint64_t p = (i + 1) << sh;
                b = b < p ? b : p;
            }
            if (a >= b) return false;
        } else if (l == 0) {
            return false;
        }
    }
}

}  // namespace pm
