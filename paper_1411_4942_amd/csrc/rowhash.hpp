// Row hash: a per-row open-addressing set of each row's columns, for the
// adjacency tests of the samplers ("is b a neighbour of a?").
//
// Row a with degree d owns the 2d entries H[2 off[a], 2 off[a+1]) (load 1/2);
// column b of the row sits at the first empty entry at or after its home
// position (linear probing, wrapping at the end of the row's entries).  A
// test reads the aligned 16 bytes that hold the home position (one line) and
// almost always ends there: at the key, or at an empty entry.  The searched
// row's offset and degree come with the query, so a test needs no other load.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pm {

constexpr uint32_t kHashEmpty = 0xFFFFFFFFu;  // not a vertex id (n < 2^31)
constexpr int64_t kHashPad = 8;              // entries after the last row (window loads)
// the build takes rows up to this degree many per block, longer rows in
// windows (the row classes of the preparation's row build bound it too)
constexpr int kHashSmallBound = 1024;
// the parts of the build: the rows of degree <= kHashSmallBound (with the
// padding after the last row), the longer rows
constexpr int kRowHashSmall = 1, kRowHashWide = 2;

// MurmurHash3's 32-bit finalizer (Appleby, public domain): spreads the bits
// of a column id over the word.
__host__ __device__ __forceinline__ uint32_t hash_mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// home position of key b in a row of `size` entries: the high word of
// mix(b) * size (Lemire's multiply-shift range reduction, no division)
__host__ __device__ __forceinline__ uint32_t hash_home(uint32_t b, uint32_t size)
{
    return (uint32_t)(((uint64_t)hash_mix32(b) * size) >> 32);
}

// Is key in the row whose slots are [lo, lo + d)?  H holds the row hash.
__host__ __device__ __forceinline__ bool rowhash_contains(const uint32_t *__restrict__ H, uint32_t lo, uint32_t d,
                                                          uint32_t key)
{
    if (d == 0) return false;
    const uint64_t base = 2ull * lo, end = base + 2ull * d;
    uint64_t cur = base + hash_home(key, 2u * d);
    // a row's entries always keep an empty one (load 1/2), so the walk ends
    // within 2d entries
    for (uint64_t seen = 0; seen < 2ull * d;) {
        const uint64_t a4 = cur & ~3ull;
        const uint4 w = *reinterpret_cast<const uint4 *>(H + a4);
        const uint32_t e[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t idx = a4 + (uint64_t)j;
            if (idx < cur || idx >= end) continue;  // before the walk, or past the row
            if (e[j] == key) return true;
            if (e[j] == kHashEmpty) return false;
            ++seen;
        }
        cur = a4 + 4;
        if (cur >= end) cur = base;  // wrap to the row's first entry
    }
    return false;
}

}  // namespace pm
