// Draw-order sort: the positions [0, kc) of a sort chunk ordered by a key of
// at most 24 bits that a functor computes from the position (the top bits of
// the sample's first draw).  The samplers' tallies are sums over sample ids,
// so the order of equal keys is free and no step needs to be stable.
//
// Two levels instead of a least-significant-digit radix sort's passes: the
// key's high digit (up to 11 bits, 2048 buckets) by one counting scatter,
// then every bucket by the low digit (up to 13 bits) in a block of its own.
//   1. keys: each tile of kDsTile positions computes its keys, stores them and
//      writes its bucket counts as one contiguous row;
//   2. column scan: each bucket's counts scanned in tile order, and the
//      bucket's total;
//   3. scatter: each tile scans the bucket totals (every bucket's first
//      position) and its own counts, groups its positions by bucket in LDS
//      and writes each bucket's run contiguously, as (low digit | position
//      << 32);
//   4. bucket sort: one block per bucket counts the low digits in LDS, scans
//      the counts, orders the positions in LDS and writes them out.
// Keys of at most 11 bits have no low digit: step 3 then writes the positions
// themselves and step 4 is skipped.
#pragma once

#include <algorithm>
#include <string>

#include "common.hpp"
#include "profile.hpp"

namespace pm {

constexpr int kDsBucketBits = 11;
constexpr int kDsBuckets = 1 << kDsBucketBits;  // high-digit buckets
constexpr int kDsLowBits = 13;                  // the widest low digit (24-bit keys)
constexpr int kDsThreads = 1024;                // keys and scatter blocks
constexpr int kDsItems = 16;                    // positions per thread there
constexpr int64_t kDsTile = (int64_t)kDsThreads * kDsItems;
constexpr int kDsScanBuckets = 16;    // buckets per column-scan block
constexpr int kDsScanParts = kWave;   // tile ranges per bucket there
constexpr int kDsScanRows = 16;       // tiles per range, at most
constexpr int64_t kDsMaxTiles = (int64_t)kDsScanParts * kDsScanRows;
// bucket-sort block and pairs per thread there (1024 x 16 measured fastest
// of 1024 x 16, 512 x 32 and 256 x 64)
constexpr int kDsSortThreads = 1024;
constexpr int kDsSortItems = 16;
constexpr uint32_t kDsSub = (uint32_t)kDsSortThreads * kDsSortItems;  // buckets ordered in LDS, at most
static_assert(kDsSub < 65536, "the counts of a bucket ordered in LDS fit 16 bits");
static_assert(kDsThreads * 2 == kDsBuckets, "the scatter block scans the buckets two per thread");
static_assert(kDsBuckets % kDsScanBuckets == 0, "whole column-scan blocks");
static_assert(kDsTile <= 65536, "tile positions fit 16 bits");

// Device buffers of one sort chunk of up to `chunk` positions, carved from one
// allocation of draw_sort_bytes(chunk) bytes.
struct DrawSortBufs {
    uint32_t *keys;    // [chunk] the keys
    uint64_t *pairs;   // [chunk] bucketed (low digit | position << 32)
    uint32_t *ids;     // [chunk] the sorted positions
    uint32_t *counts;  // [tiles][kDsBuckets] per-tile bucket counts
    uint32_t *colpre;  // [tiles][kDsBuckets] each tile's start inside each bucket
    uint32_t *totals;  // [kDsBuckets] bucket sizes
    uint32_t *bstart;  // [kDsBuckets + 1] bucket starts, then the chunk size
    uint64_t chunk;
};

constexpr int64_t draw_sort_tiles(uint64_t chunk)
{
    return chunk == 0 ? 1 : ((int64_t)chunk + kDsTile - 1) / kDsTile;
}

constexpr size_t ds_align(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr size_t draw_sort_bytes(uint64_t chunk)
{
    return ds_align(4 * chunk) + ds_align(8 * chunk) + ds_align(4 * chunk) +
           2 * ds_align(4 * (size_t)draw_sort_tiles(chunk) * kDsBuckets) + ds_align(4 * kDsBuckets) +
           ds_align(4 * (kDsBuckets + 1));
}

// base: device memory of draw_sort_bytes(chunk) bytes, 256-byte aligned
inline void draw_sort_carve(void *base, uint64_t chunk, DrawSortBufs *b)
{
    const size_t tiles = (size_t)draw_sort_tiles(chunk);
    char *p = (char *)base;
    b->keys = (uint32_t *)p;
    p += ds_align(4 * chunk);
    b->pairs = (uint64_t *)p;
    p += ds_align(8 * chunk);
    b->ids = (uint32_t *)p;
    p += ds_align(4 * chunk);
    b->counts = (uint32_t *)p;
    p += ds_align(4 * tiles * kDsBuckets);
    b->colpre = (uint32_t *)p;
    p += ds_align(4 * tiles * kDsBuckets);
    b->totals = (uint32_t *)p;
    p += ds_align(4 * kDsBuckets);
    b->bstart = (uint32_t *)p;
    b->chunk = chunk;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2: the
// scatter gives every XCD a contiguous run of tiles, so that the runs which
// neighbouring tiles write side by side inside a bucket meet in one L2.
__device__ __forceinline__ int64_t ds_xcd_tile(int64_t b, int64_t nb)
{
    constexpr int64_t kX = 8;
    const int64_t x = b % kX, i = b / kX;
    const int64_t per = nb / kX, extra = nb % kX;
    return x * per + (x < extra ? x : extra) + i;
}

// exclusive prefix of v over the block's threads (whole waves; s_w holds one
// word per wave and is not reused before the block synchronises again)
template <int THREADS>
__device__ __forceinline__ uint32_t ds_block_excl(uint32_t v, uint32_t *s_w)
{
    const int lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int ww = 0; ww < THREADS / kWave; ++ww)
        if (ww < w) pre += s_w[ww];
    return pre + incl - v;
}

template <class KeyFn>
static __global__ __launch_bounds__(kDsThreads) void ds_keys(KeyFn kf, int64_t kc, int hshift,
                                                           uint32_t *__restrict__ keys,
                                                           uint32_t *__restrict__ counts)
{
    __shared__ uint32_t hist[kDsBuckets];
    const int t = threadIdx.x;
    for (int b = t; b < kDsBuckets; b += kDsThreads) hist[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kDsTile;
    for (int i = 0; i < kDsItems; ++i) {
        const int64_t pos = base + (int64_t)i * kDsThreads + t;
        if (pos < kc) {
            const uint32_t key = kf(pos);
            keys[pos] = key;
            atomicAdd(&hist[(key >> hshift) & (kDsBuckets - 1)], 1u);
        }
    }
    __syncthreads();
    for (int b = t; b < kDsBuckets; b += kDsThreads) counts[(int64_t)blockIdx.x * kDsBuckets + b] = hist[b];
}

// Block b covers buckets [16 b, 16 b + 16): thread (p, j) sums bucket
// 16 b + j over the tiles [p per, (p + 1) per) (per <= kDsScanRows; a row
// read is 64 contiguous bytes), keeping its counts in registers; wave j then
// scans bucket 16 b + j's 64 part sums across its lanes, and each thread
// rewrites its tiles' counts as starts.
static __global__ __launch_bounds__(kDsScanBuckets *kDsScanParts) void ds_colscan(
    const uint32_t *__restrict__ counts, int64_t tiles, uint32_t *__restrict__ colpre, uint32_t *__restrict__ totals)
{
    static_assert(kDsScanParts == kWave && kDsScanBuckets * kDsScanParts / kWave == kDsScanBuckets,
                  "one wave per bucket scans its parts");
    __shared__ uint32_t s_part[kDsScanParts][kDsScanBuckets + 1];
    const int j = threadIdx.x % kDsScanBuckets, p = threadIdx.x / kDsScanBuckets;
    const uint32_t b = blockIdx.x * kDsScanBuckets + j;
    const uint32_t nt = (uint32_t)tiles;
    const uint32_t per = (nt + kDsScanParts - 1) / kDsScanParts;  // <= kDsScanRows (checked by the host)
    const uint32_t t0 = std::min<uint32_t>(p * per, nt), t1 = std::min<uint32_t>(t0 + per, nt);
    uint32_t v[kDsScanRows];
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kDsScanRows; ++i) {
        v[i] = (t0 + i < t1) ? counts[(t0 + i) * kDsBuckets + b] : 0u;
        acc += v[i];
    }
    s_part[p][j] = acc;
    __syncthreads();
    {
        // wave w: bucket 16 b + w, lane q: part q
        const int w = threadIdx.x / kWave, q = lane_id();
        const uint32_t x = s_part[q][w];
        uint32_t incl = x;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(incl, d, kWave);
            if (q >= d) incl += o;
        }
        s_part[q][w] = incl - x;
        if (q == kWave - 1) totals[blockIdx.x * kDsScanBuckets + w] = incl;
    }
    __syncthreads();
    uint32_t run = s_part[p][j];
#pragma unroll
    for (int i = 0; i < kDsScanRows; ++i)
        if (t0 + i < t1) {
            colpre[(t0 + i) * kDsBuckets + b] = run;
            run += v[i];
        }
}

// The tile's positions grouped by bucket in LDS (an LDS atomic per position
// on the tile's own bucket starts), then written out in LDS order: the run of
// each bucket goes to consecutive addresses.  With hshift == 0 the positions
// go straight to ids (the buckets are the keys); otherwise (low digit |
// position << 32) goes to pairs.
static __global__ __launch_bounds__(kDsThreads) void ds_scatter(const uint32_t *__restrict__ keys, int64_t kc,
                                                              int hshift, const uint32_t *__restrict__ counts,
                                                              const uint32_t *__restrict__ colpre,
                                                              const uint32_t *__restrict__ totals, int64_t tiles,
                                                              uint64_t *__restrict__ pairs,
                                                              uint32_t *__restrict__ ids,
                                                              uint32_t *__restrict__ bstart)
{
    __shared__ uint32_t s_key[kDsTile];
    __shared__ uint16_t s_pos[kDsTile];
    __shared__ uint32_t s_cur[kDsBuckets];    // the tile's next free LDS slot of each bucket
    __shared__ uint32_t s_delta[kDsBuckets];  // output position minus LDS slot, per bucket
    __shared__ uint32_t s_w0[kDsThreads / kWave], s_w1[kDsThreads / kWave];
    const int t = threadIdx.x;
    const int64_t tile = ds_xcd_tile(blockIdx.x, tiles);
    const int64_t base = tile * kDsTile;
    const int tile_n = (int)std::min<int64_t>(kDsTile, kc - base);
    // the tile's keys, all loads in flight before the scans
    uint32_t key[kDsItems];
#pragma unroll
    for (int i = 0; i < kDsItems; ++i) {
        const int idx = i * kDsThreads + t;
        key[i] = idx < tile_n ? keys[base + idx] : 0u;
    }
    // two buckets per thread: the buckets' first output positions (totals
    // scanned) and the tile's own bucket starts (its counts scanned)
    const uint2 tot = reinterpret_cast<const uint2 *>(totals)[t];
    const uint2 own = reinterpret_cast<const uint2 *>(counts + tile * kDsBuckets)[t];
    const uint2 pre = reinterpret_cast<const uint2 *>(colpre + tile * kDsBuckets)[t];
    const uint32_t g0 = ds_block_excl<kDsThreads>(tot.x + tot.y, s_w0);
    const uint32_t l0 = ds_block_excl<kDsThreads>(own.x + own.y, s_w1);
    {
        const int b = 2 * t;
        const uint32_t g1 = g0 + tot.x, l1 = l0 + own.x;
        s_cur[b] = l0;
        s_cur[b + 1] = l1;
        s_delta[b] = g0 + pre.x - l0;
        s_delta[b + 1] = g1 + pre.y - l1;
        if (blockIdx.x == 0) {
            bstart[b] = g0;
            bstart[b + 1] = g1;
            if (t == 0) bstart[kDsBuckets] = (uint32_t)kc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kDsItems; ++i) {
        const int idx = i * kDsThreads + t;
        if (idx < tile_n) {
            const uint32_t at = atomicAdd(&s_cur[(key[i] >> hshift) & (kDsBuckets - 1)], 1u);
            if (at < (uint32_t)tile_n) {  // always: the counts were taken from the same keys
                s_key[at] = key[i];
                s_pos[at] = (uint16_t)idx;
            }
        }
    }
    __syncthreads();
    const uint32_t lomask = (1u << hshift) - 1u;
#pragma unroll
    for (int i = 0; i < kDsItems; ++i) {
        const int j = i * kDsThreads + t;
        if (j < tile_n) {
            const uint32_t k = s_key[j];
            const uint32_t dst = (uint32_t)j + s_delta[(k >> hshift) & (kDsBuckets - 1)];
            const uint32_t pos = (uint32_t)base + s_pos[j];
            if (dst < (uint32_t)kc) {  // always: the bucket starts come from the same counts
                if (hshift == 0)
                    ids[dst] = pos;
                else
                    pairs[dst] = (uint64_t)(k & lomask) | ((uint64_t)pos << 32);
            }
        }
    }
}

// One block per bucket: a counting sort on the low digit (lobits <= 13).  A
// bucket of at most kDsSub positions is read once (all loads issued before
// the LDS atomics) and kept in registers, counted with two 16-bit counters
// per word, ordered in LDS and written out contiguously.  A larger bucket
// (keys bunched into few buckets, or chunks near 2^24 samples) is counted
// with 32-bit counters in the staging space, batch by batch, and its
// positions written in place.
static __global__ __launch_bounds__(kDsSortThreads) void ds_bucket_sort(const uint64_t *__restrict__ pairs,
                                                                      const uint32_t *__restrict__ bstart,
                                                                      int lobits, uint32_t *__restrict__ ids)
{
    // 80 KiB in all, so that two blocks share a CU's 160 KiB: the block-scan
    // words live in the staging space, which holds nothing during the scan
    __shared__ uint32_t cnt[1 << (kDsLowBits - 1)];
    __shared__ uint32_t s_ids[kDsSub];  // the staging space (32-bit counters of a large bucket)
    static_assert(kDsSub >= (1u << kDsLowBits) + kDsSortThreads / kWave,
                  "a large bucket's counters and the scan words fit the staging space");
    const int t = threadIdx.x;
    const uint32_t lo = bstart[blockIdx.x], hi = bstart[blockIdx.x + 1];
    if (hi <= lo + 1) {  // the block's bounds are uniform: nothing to order
        if (hi == lo + 1 && t == 0) ids[lo] = (uint32_t)(pairs[lo] >> 32);
        return;
    }
    const uint32_t n = hi - lo;
    const uint32_t lomask = (1u << lobits) - 1u;
    uint64_t pr[kDsSortItems];
    if (n <= kDsSub) {
        const int nw = 1 << (lobits - 1);  // counter words
        for (int w = t; w < nw; w += kDsSortThreads) cnt[w] = 0;
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i) {
            const uint32_t e = (uint32_t)(i * kDsSortThreads + t);
            pr[i] = e < n ? pairs[lo + e] : ~0ull;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i)
            if (pr[i] != ~0ull) {
                const uint32_t d = (uint32_t)pr[i] & lomask;
                atomicAdd(&cnt[d >> 1], 1u << ((d & 1u) << 4));
            }
        __syncthreads();
        // each thread a run of counter words: the sum of its digits, the
        // block's exclusive prefix, then the run rewritten as starts (a
        // thread touches only its own run)
        const int per = (nw + kDsSortThreads - 1) / kDsSortThreads;
        const int w0 = std::min(t * per, nw), w1 = std::min(w0 + per, nw);
        uint32_t sum = 0;
        for (int w = w0; w < w1; ++w) {
            const uint32_t x = cnt[w];
            sum += (x & 0xFFFFu) + (x >> 16);
        }
        uint32_t run = ds_block_excl<kDsSortThreads>(sum, s_ids);  // staging still empty
        for (int w = w0; w < w1; ++w) {
            const uint32_t x = cnt[w];
            const uint32_t a = run, b = run + (x & 0xFFFFu);
            cnt[w] = a | (b << 16);
            run = b + (x >> 16);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i)
            if (pr[i] != ~0ull) {
                const uint32_t d = (uint32_t)pr[i] & lomask, sh = (d & 1u) << 4;
                const uint32_t at = (atomicAdd(&cnt[d >> 1], 1u << sh) >> sh) & 0xFFFFu;
                if (at < n) s_ids[at] = (uint32_t)(pr[i] >> 32);  // always: the counts are this bucket's
            }
        __syncthreads();
        for (uint32_t j = t; j < n; j += kDsSortThreads) ids[lo + j] = s_ids[j];
        return;
    }
    uint32_t *c32 = s_ids;
    const int nlo = 1 << lobits;
    for (int d = t; d < nlo; d += kDsSortThreads) c32[d] = 0;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < n; e0 += kDsSub) {
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i) {
            const uint32_t e = e0 + (uint32_t)(i * kDsSortThreads + t);
            pr[i] = e < n ? pairs[lo + e] : ~0ull;
        }
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i)
            if (pr[i] != ~0ull) atomicAdd(&c32[(uint32_t)pr[i] & lomask], 1u);
    }
    __syncthreads();
    const int per = (nlo + kDsSortThreads - 1) / kDsSortThreads;
    const int d0 = std::min(t * per, nlo), d1 = std::min(d0 + per, nlo);
    uint32_t sum = 0;
    for (int d = d0; d < d1; ++d) sum += c32[d];
    uint32_t run = ds_block_excl<kDsSortThreads>(sum, s_ids + (1 << kDsLowBits));  // past the counters
    for (int d = d0; d < d1; ++d) {
        const uint32_t x = c32[d];
        c32[d] = run;
        run += x;
    }
    __syncthreads();
    for (uint32_t e0 = 0; e0 < n; e0 += kDsSub) {
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i) {
            const uint32_t e = e0 + (uint32_t)(i * kDsSortThreads + t);
            pr[i] = e < n ? pairs[lo + e] : ~0ull;
        }
#pragma unroll
        for (int i = 0; i < kDsSortItems; ++i)
            if (pr[i] != ~0ull) {
                const uint32_t at = atomicAdd(&c32[(uint32_t)pr[i] & lomask], 1u);
                if (at < n) ids[lo + at] = (uint32_t)(pr[i] >> 32);  // always: the counts are this bucket's
            }
    }
}

// Sort the positions [0, kc) of a chunk by kf(position) < 2^kbits (1 <= kbits
// <= 24, 1 <= kc <= b.chunk, at most kDsMaxTiles tiles), on stream s; *ids
// receives b.ids.
template <class KeyFn>
pm_status draw_sort(const char *name, KeyFn kf, uint64_t kc, int kbits, hipStream_t s, const DrawSortBufs &b,
                    uint32_t **ids)
{
    if (kc == 0 || kc > b.chunk || draw_sort_tiles(kc) > kDsMaxTiles || kbits < 1 ||
        kbits > kDsBucketBits + kDsLowBits) {
        set_error(std::string(name) + ": chunk size or key width out of range");
        return PM_EINVAL;
    }
    const int hshift = kbits > kDsBucketBits ? kbits - kDsBucketBits : 0;
    const int64_t tiles = draw_sort_tiles(kc);
    // the scopes keep their names until they end
    const std::string n_keys = std::string(name) + ".keys", n_scan = std::string(name) + ".colscan",
                      n_scat = std::string(name) + ".scatter", n_buck = std::string(name) + ".buckets";
    {
        ProfScope p(n_keys.c_str(), s);
        hipLaunchKernelGGL((ds_keys<KeyFn>), dim3((unsigned)tiles), dim3(kDsThreads), 0, s, kf, (int64_t)kc, hshift,
                           b.keys, b.counts);
        PM_HIP(hipGetLastError());
    }
    {
        ProfScope p(n_scan.c_str(), s);
        hipLaunchKernelGGL(ds_colscan, dim3(kDsBuckets / kDsScanBuckets), dim3(kDsScanBuckets * kDsScanParts), 0, s,
                           b.counts, tiles, b.colpre, b.totals);
        PM_HIP(hipGetLastError());
    }
    {
        ProfScope p(n_scat.c_str(), s);
        hipLaunchKernelGGL(ds_scatter, dim3((unsigned)tiles), dim3(kDsThreads), 0, s, b.keys, (int64_t)kc, hshift,
                           b.counts, b.colpre, b.totals, tiles, b.pairs, b.ids, b.bstart);
        PM_HIP(hipGetLastError());
    }
    if (hshift > 0) {
        ProfScope p(n_buck.c_str(), s);
        hipLaunchKernelGGL(ds_bucket_sort, dim3(kDsBuckets), dim3(kDsSortThreads), 0, s, b.pairs, b.bstart, hshift,
                           b.ids);
        PM_HIP(hipGetLastError());
    }
    *ids = b.ids;
    return PM_OK;
}

}  // namespace pm
