// Wave-cooperative membership search over the ladder index (device only;
// ladder.hpp holds the per-lane search, which also builds for the host).
#pragma once

#include "ladder.hpp"

namespace pm {

// Wave-cooperative form of ladder_contains: each lane brings one query (a row
// window [lo, hi) and a key; `active` false for none) and gets its answer.
// Every level of every query reads the same 128-byte line as the per-lane
// search, but the wave reads it cooperatively: half a wave (32 lanes x 4
// bytes) loads one query's line in a single coalesced request, two queries per
// load instruction, and a ballot counts the entries <= key inside the query's
// window.  The per-lane form issues eight 16-byte loads per lane per line.
// Must be called by all 64 lanes of the wave together (wave-uniform control
// flow); lanes without a query pass active = false.
__device__ __forceinline__ bool ladder_contains_wave(const Ladder &L, bool active, uint32_t lo, uint32_t hi,
                                                     uint32_t key)
{
    const uint32_t lane = __lane_id();
    const uint32_t half = lane >> 5, sub = lane & 31u;
    bool live = active && lo < hi;
    bool found = false;
    int l = 0;
    if (live) {
        while (l < L.top) {  // lowest level whose samples inside [lo, hi) share one line
            const uint32_t sh = 5u * l;
            const uint64_t a = ((uint64_t)lo + (1ull << sh) - 1) >> sh, b = (uint64_t)(hi - 1) >> sh;
            if (a > b || (a >> 5) == (b >> 5)) break;
            ++l;
        }
    }
    uint64_t a = lo, b = hi;  // slot window holding the last entry <= key
    while (__ballot(live) != 0ull) {
        // this round's line, and the window [j0, j1] of the level's samples in it
        const uint32_t *line = nullptr;
        uint32_t win = 0;  // j0 | j1 << 8
        bool need = false;
        uint64_t first = 0;
        if (live) {
            const uint32_t sh = 5u * l;
            first = (a + (1ull << sh) - 1) >> sh;
            const uint64_t last = (b - 1) >> sh;
            if (first <= last) {
                const uint64_t cell = first >> 5;
                line = L.lvl[l] + cell * 32;
                win = (uint32_t)(first - cell * 32) | ((uint32_t)(last - cell * 32) << 8);
                need = true;
            }
        }
        const uint64_t needm = __ballot(need);
        const uint64_t lp = (uint64_t)(uintptr_t)line;
        const uint32_t lp_lo = (uint32_t)lp, lp_hi = (uint32_t)(lp >> 32);
        uint32_t cnt = 0;
        bool eq_mine = false;
        // every pair's line first (all loads of the round in flight), then
        // the comparisons
        uint32_t w[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            w[q] = 0;
            if ((needm >> (2 * q)) & 3ull) {  // wave-uniform
                const uint32_t e = 2 * q, o = 2 * q + 1;
                const uint32_t plo = half ? __builtin_amdgcn_readlane(lp_lo, o) : __builtin_amdgcn_readlane(lp_lo, e);
                const uint32_t phi = half ? __builtin_amdgcn_readlane(lp_hi, o) : __builtin_amdgcn_readlane(lp_hi, e);
                if ((needm >> (half ? o : e)) & 1ull)
                    w[q] = reinterpret_cast<const uint32_t *>((uintptr_t)plo | ((uint64_t)phi << 32))[sub];
            }
        }
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if ((needm >> (2 * q)) & 3ull) {  // wave-uniform
                const uint32_t e = 2 * q, o = 2 * q + 1;
                const uint32_t k = half ? __builtin_amdgcn_readlane(key, o) : __builtin_amdgcn_readlane(key, e);
                const uint32_t wn = half ? __builtin_amdgcn_readlane(win, o) : __builtin_amdgcn_readlane(win, e);
                const bool ld = (needm >> (half ? o : e)) & 1ull;
                const bool in = ld && sub >= (wn & 0xFFu) && sub <= (wn >> 8);
                const uint64_t le = __ballot(in && w[q] <= k);
                const uint64_t eq = __ballot(in && w[q] == k);
                if (lane == e) {
                    cnt = (uint32_t)__popcll(le & 0xFFFFFFFFull);
                    eq_mine = (eq & 0xFFFFFFFFull) != 0;
                } else if (lane == o) {
                    cnt = (uint32_t)__popcll(le >> 32);
                    eq_mine = (eq >> 32) != 0;
                }
            }
        }
        if (live) {
            const uint32_t sh = 5u * l;
            if (need) {
                if (eq_mine) {
                    found = true;
                    live = false;
                } else if (l == 0) {
                    live = false;
                } else {
                    if (cnt == 0) {
                        const uint64_t p = first << sh;
                        b = b < p ? b : p;
                    } else {
                        const uint64_t i = first + cnt - 1;
                        a = i << sh;
                        const uint64_t p = (i + 1) << sh;
                        b = b < p ? b : p;
                    }
                    if (a >= b) live = false;
                    --l;
                }
            } else if (l == 0) {
                live = false;
            } else {
                --l;
            }
        }
    }
    return found;
}

}  // namespace pm
