// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits.
//
// One pass: per-tile digit histograms (tile-major layout: each tile's 256
// counts are one contiguous kilobyte, written and read whole), their
// exclusive scan in digit-major order (per-chunk sums, one scan block, and a
// rewrite of the chunks into offsets), and a stable scatter.  The scatter ranks
// each wave's 1024 elements in input order with ballots (8 ballots give every
// lane the mask of lanes holding the same digit) and per-wave digit counters
// in LDS, combines the four waves per digit, stages the tile digit-sorted in
// LDS, then writes each digit run contiguously.
#pragma once

#include <string>

#include "profile.hpp"
#include "scan.hpp"

namespace pm {

// The kernels have internal linkage: each translation unit that sorts keeps
// its own copy.

#ifndef PM_RADIX_THREADS
#define PM_RADIX_THREADS 512
#endif
constexpr int kRadixThreads = PM_RADIX_THREADS;  // threads per histogram / scatter block (512 measured fastest of 256, 512, 1024)
constexpr int kRadixWaves = kRadixThreads / kWave;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;
constexpr int kRadixBins = 256;
static_assert(kRadixThreads >= kRadixBins && kRadixThreads % kRadixBins == 0, "one thread per digit, whole waves");

// Tile layout shared by both kernels: wave w owns elements
// [w * 1024, (w + 1) * 1024) of the tile, as 16 coalesced rows of 64, so the
// element order inside a tile is (wave, row, lane).  Threads t < 256 also
// stand for digit t in the per-digit phases.
constexpr int kRadixWaveSpan = kWave * kRadixItems;  // 1024

__device__ __forceinline__ int64_t radix_index(int64_t tile, int w, int i, int lane)
{
    return tile * kRadixTile + (int64_t)w * kRadixWaveSpan + (int64_t)i * kWave + lane;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  Give
// every XCD a contiguous run of tiles so that the digit runs that neighbouring
// tiles write next to each other meet in the same L2 and leave it as whole
// lines.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb)
{
    const int64_t x = b % kXcds, i = b / kXcds;
    const int64_t per = nb / kXcds, extra = nb % kXcds;
    return x * per + (x < extra ? x : extra) + i;
}

// Digit counts of one tile.  Four LDS histograms per wave (lane & 3 picks
// one) quarter the atomic conflicts of skewed digits (R-MAT's high column
// bits); the copies are summed at the end.
constexpr int kHistCopies = 4;

static __global__ __launch_bounds__(kRadixThreads) void radix_histogram(const uint32_t *__restrict__ keys, int64_t N,
                                                                  int shift, uint32_t mask,
                                                                  uint32_t *__restrict__ counts, int64_t tiles)
{
    __shared__ uint32_t hist[kRadixWaves * kHistCopies][kRadixBins];
    const int t = threadIdx.x, w0 = t / kWave, lane = lane_id();
    const int w = w0 * kHistCopies + (lane & (kHistCopies - 1));  // this lane's histogram copy
    for (int j = t; j < kRadixWaves * kHistCopies * kRadixBins; j += kRadixThreads) (&hist[0][0])[j] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blockIdx.x * kRadixTile;
    if (tile0 + kRadixTile <= N && ((uintptr_t)keys & 15u) == 0) {
        // whole tile: counting ignores order, so each lane takes 16-byte loads
        const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + tile0 + (int64_t)w0 * kRadixWaveSpan);
        uint4 v[kRadixItems / 4];
#pragma unroll
        for (int q = 0; q < kRadixItems / 4; ++q) v[q] = k4[q * kWave + lane];
#pragma unroll
        for (int q = 0; q < kRadixItems / 4; ++q) {
            atomicAdd(&hist[w][(v[q].x >> shift) & mask], 1u);
            atomicAdd(&hist[w][(v[q].y >> shift) & mask], 1u);
            atomicAdd(&hist[w][(v[q].z >> shift) & mask], 1u);
            atomicAdd(&hist[w][(v[q].w >> shift) & mask], 1u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kRadixItems; ++i) {
            int64_t idx = radix_index(blockIdx.x, w0, i, lane);
            if (idx < N) atomicAdd(&hist[w][(keys[idx] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    if (t < kRadixBins) {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kRadixWaves * kHistCopies; ++i) c += hist[i][t];
        counts[(int64_t)blockIdx.x * kRadixBins + t] = c;
    }
}

// vals_in may be null: the payload is then the element's input position.
// keys_out may be null: with pair_out given, pair_out[dst] = key | val << 32
// replaces the key array; without, the keys are not written (vals_out is
// always written).
// sample_out, when given, receives every 32nd value: sample_out[dst / 32].
static __global__ __launch_bounds__(kRadixThreads) void radix_scatter(const uint32_t *__restrict__ keys_in,
                                                        const uint32_t *__restrict__ vals_in, int64_t N, int shift,
                                                        uint32_t mask, const uint32_t *__restrict__ offsets,
                                                        int64_t tiles, uint32_t *__restrict__ keys_out,
                                                        uint32_t *__restrict__ vals_out,
                                                        uint64_t *__restrict__ pair_out,
                                                        uint32_t *__restrict__ sample_out)
{
    __shared__ uint32_t s_key[kRadixTile];
    __shared__ uint32_t s_val[kRadixTile];
    __shared__ uint32_t s_cnt[kRadixWaves][kRadixBins];  // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_start[kRadixBins];             // first LDS slot of each digit in the tile
    __shared__ uint32_t s_goff[kRadixBins];              // first output position of each digit
    __shared__ uint32_t s_wsum[kRadixBins / kWave];

    const int t = threadIdx.x;
    const int w = t / kWave;
    const int lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t tile = xcd_tile(blockIdx.x, tiles);

    for (int j = t; j < kRadixWaves * kRadixBins; j += kRadixThreads) (&s_cnt[0][0])[j] = 0;
    if (t < kRadixBins) s_goff[t] = offsets[tile * kRadixBins + t];

    uint32_t key[kRadixItems], val[kRadixItems], dig[kRadixItems], rank[kRadixItems];
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        int64_t idx = radix_index(tile, w, i, lane);
        bool ok = idx < N;
        key[i] = ok ? keys_in[idx] : 0u;
        val[i] = ok ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
        dig[i] = (key[i] >> shift) & mask;
    }
    __syncthreads();

    // stable rank inside the wave's 1024 elements: lanes holding the same
    // digit find each other with 8 ballots; the group's lowest lane bumps the
    // wave's counter for that digit (one wave: LDS reads precede the write)
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        int64_t idx = radix_index(tile, w, i, lane);
        bool ok = idx < N;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((dig[i] >> b) & 1u);
            peers &= ((dig[i] >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = __popcll(peers & lt_mask);
        const uint32_t base = s_cnt[w][dig[i]];
        rank[i] = base + below;
        if (ok && below == 0) s_cnt[w][dig[i]] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();

    // per digit (threads t < 256, whole waves): the tile's digit totals,
    // scanned over digits, and each wave's start inside its digit's run
    uint32_t total = 0, incl = 0;
    if (t < kRadixBins) {
#pragma unroll
        for (int i = 0; i < kRadixWaves; ++i) total += s_cnt[i][t];
        incl = total;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            uint32_t o = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += o;
        }
        if (lane == kWave - 1) s_wsum[w] = incl;
    }
    __syncthreads();
    if (t < kRadixBins) {
        uint32_t pre = 0;
        for (int ww = 0; ww < w; ++ww) pre += s_wsum[ww];
        s_start[t] = pre + incl - total;
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < kRadixWaves; ++i) {
            const uint32_t c = s_cnt[i][t];
            s_cnt[i][t] = run;
            run += c;
        }
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        int64_t idx = radix_index(tile, w, i, lane);
        if (idx < N) {
            uint32_t pos = s_start[dig[i]] + s_cnt[w][dig[i]] + rank[i];
            s_key[pos] = key[i];
            s_val[pos] = val[i];
        }
    }
    __syncthreads();

    const int64_t tile_n = (N - tile * kRadixTile) < kRadixTile ? (N - tile * kRadixTile) : kRadixTile;
#pragma unroll
    for (int i = 0; i < kRadixItems; ++i) {
        int p = i * kRadixThreads + t;
        if (p < tile_n) {
            uint32_t k = s_key[p];
            uint32_t d = (k >> shift) & mask;
            uint32_t dst = s_goff[d] + (uint32_t)(p - s_start[d]);
            const uint32_t vv = s_val[p];
            if (pair_out)
                pair_out[dst] = (uint64_t)k | ((uint64_t)vv << 32);
            else if (keys_out)
                keys_out[dst] = k;
            vals_out[dst] = vv;
            if (sample_out && (dst & 31u) == 0) sample_out[dst >> 5] = vv;
        }
    }
}

// Exclusive scan of the tile-major counts in (digit, tile) order: the output
// position of digit d of tile t is the number of keys with a smaller digit
// plus those with digit d in earlier tiles.  Tiles are grouped in chunks of
// kRadixChunk; thread d of a block handles digit d, reading one contiguous
// row of 256 counts per tile.
constexpr int kRadixChunk = 64;
constexpr int kRadixBatch = 8;  // loads in flight per thread
constexpr int kRadixParts = 4;  // threads per digit in the chunk scan

static __global__ __launch_bounds__(kBlock) void radix_chunk_sums(const uint32_t *__restrict__ counts, int64_t tiles,
                                                           uint32_t *__restrict__ chunk)
{
    const int d = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kRadixChunk;
    const int64_t t1 = (t0 + kRadixChunk < tiles) ? t0 + kRadixChunk : tiles;
    uint32_t acc = 0;
    for (int64_t t = t0; t < t1; t += kRadixBatch) {
        uint32_t v[kRadixBatch];
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) v[i] = (t + i < t1) ? counts[(t + i) * kRadixBins + d] : 0u;
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) acc += v[i];
    }
    chunk[(int64_t)blockIdx.x * kRadixBins + d] = acc;
}

// One block of kRadixParts * 256 threads: thread (p, d) owns a contiguous
// range of chunks of digit d.  chunk[c][d] becomes the output position of
// digit d's first key in chunk c.
static __global__ __launch_bounds__(kRadixParts *kBlock) void radix_chunk_scan(uint32_t *__restrict__ chunk,
                                                                        int64_t nchunks)
{
    __shared__ uint32_t s_part[kRadixParts][kRadixBins];
    __shared__ uint32_t s_wave[kBlock / kWave];
    const int d = threadIdx.x % kRadixBins, p = threadIdx.x / kRadixBins;
    const int64_t per = (nchunks + kRadixParts - 1) / kRadixParts;
    const int64_t c0 = p * per, c1 = (c0 + per < nchunks) ? c0 + per : nchunks;
    uint32_t acc = 0;
    for (int64_t c = c0; c < c1; c += kRadixBatch) {
        uint32_t v[kRadixBatch];
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) v[i] = (c + i < c1) ? chunk[(c + i) * kRadixBins + d] : 0u;
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) acc += v[i];
    }
    s_part[p][d] = acc;
    __syncthreads();
    // digit totals, exclusive over digits (the threads of part 0, whole waves)
    const int lane = lane_id(), w = d / kWave;
    uint32_t tot = 0, incl = 0;
    if (p == 0) {
#pragma unroll
        for (int q = 0; q < kRadixParts; ++q) tot += s_part[q][d];
        incl = tot;
#pragma unroll
        for (int k = 1; k < kWave; k <<= 1) {
            const uint32_t o = __shfl_up(incl, k, kWave);
            if (lane >= k) incl += o;
        }
        if (lane == kWave - 1) s_wave[w] = incl;
    }
    __syncthreads();
    if (p == 0) {
        uint32_t pre = 0;
        for (int ww = 0; ww < w; ++ww) pre += s_wave[ww];
        // the digit's base, then each part's start within the digit
        uint32_t run = pre + incl - tot;
#pragma unroll
        for (int q = 0; q < kRadixParts; ++q) {
            const uint32_t x = s_part[q][d];
            s_part[q][d] = run;
            run += x;
        }
    }
    __syncthreads();
    uint32_t run = s_part[p][d];
    for (int64_t c = c0; c < c1; c += kRadixBatch) {
        uint32_t v[kRadixBatch];
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) v[i] = (c + i < c1) ? chunk[(c + i) * kRadixBins + d] : 0u;
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i)
            if (c + i < c1) {
                chunk[(c + i) * kRadixBins + d] = run;
                run += v[i];
            }
    }
}

static __global__ __launch_bounds__(kBlock) void radix_chunk_apply(const uint32_t *__restrict__ counts,
                                                            const uint32_t *__restrict__ chunk, int64_t tiles,
                                                            uint32_t *__restrict__ offs)
{
    const int d = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kRadixChunk;
    const int64_t t1 = (t0 + kRadixChunk < tiles) ? t0 + kRadixChunk : tiles;
    uint32_t run = chunk[(int64_t)blockIdx.x * kRadixBins + d];
    for (int64_t t = t0; t < t1; t += kRadixBatch) {
        uint32_t v[kRadixBatch];
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i) v[i] = (t + i < t1) ? counts[(t + i) * kRadixBins + d] : 0u;
#pragma unroll
        for (int i = 0; i < kRadixBatch; ++i)
            if (t + i < t1) {
                offs[(t + i) * kRadixBins + d] = run;
                run += v[i];
            }
    }
}

// Device scratch needed by radix_sort for N elements.
inline size_t radix_scratch_bytes(int64_t N)
{
    int64_t tiles = (N + kRadixTile - 1) / kRadixTile;
    if (tiles < 1) tiles = 1;
    const int64_t cnt = tiles * kRadixBins;
    const int64_t chunks = (tiles + kRadixChunk - 1) / kRadixChunk;
    return (size_t)(2 * cnt + chunks * kRadixBins) * sizeof(uint32_t) + 1024;
}

// Sort (keys, vals) by the low `bits` bits of the keys, stably.  The first
// pass reads (in_k, in_v), which are never written (in_v null: the payload
// is the input position); passes alternate between the buffer pairs
// (k0, v0) and (k1, v1).  On return *out_k / *out_v point at the result.
// With pair_out, the last pass writes key | val << 32 there instead of the
// keys (*out_k is then null); with sample_out it also writes every 32nd
// value.  With keys_wanted false the last pass writes no keys (*out_k is
// then null).  N < 2^32.
static __global__ void radix_pair_copy(const uint32_t *__restrict__ k, const uint32_t *__restrict__ v, int64_t N,
                                uint64_t *__restrict__ pair, uint32_t *__restrict__ sample, uint32_t *__restrict__ vcopy)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t vv = v ? v[i] : (uint32_t)i;
        if (pair) pair[i] = (uint64_t)k[i] | ((uint64_t)vv << 32);
        if (sample && (i & 31) == 0) sample[i >> 5] = vv;
        vcopy[i] = vv;
    }
}

// One stable LSD sort as a sequence of 8-bit passes, enqueued one at a time
// by step() (two sorts on two streams can then be enqueued pass by pass, so
// that neither stream waits for the host to enqueue the other's passes).
// Arguments as radix_sort; N > 1 and bits > 0.
struct RadixRun {
    std::string n_hist, n_scan, n_scat;
    const uint32_t *ki, *vi;
    uint32_t *k0, *v0, *k1, *v1, *ko, *vo;
    int64_t N, tiles, chunks;
    int bits, shift = 0;
    uint32_t *counts, *offs, *chunk;
    hipStream_t s;
    uint64_t *pair_out;
    uint32_t *sample_out;
    bool keys_wanted;
    uint32_t *out_k, *out_v;

    RadixRun(const char *name, const uint32_t *in_k, const uint32_t *in_v, uint32_t *k0_, uint32_t *v0_,
             uint32_t *k1_, uint32_t *v1_, int64_t N_, int bits_, void *scratch, hipStream_t s_,
             uint64_t *pair_out_ = nullptr, uint32_t *sample_out_ = nullptr, bool keys_wanted_ = true)
        : n_hist(std::string(name) + ".histogram"), n_scan(std::string(name) + ".count_scan"),
          n_scat(std::string(name) + ".scatter"), ki(in_k), vi(in_v), k0(k0_), v0(v0_), k1(k1_), v1(v1_), ko(k0_),
          vo(v0_), N(N_), bits(bits_), s(s_), pair_out(pair_out_), sample_out(sample_out_),
          keys_wanted(keys_wanted_), out_k(k0_), out_v(v0_)
    {
        tiles = (N + kRadixTile - 1) / kRadixTile;
        chunks = (tiles + kRadixChunk - 1) / kRadixChunk;
        counts = (uint32_t *)scratch;
        offs = counts + tiles * kRadixBins;
        chunk = offs + tiles * kRadixBins;
    }
    bool done() const { return shift >= bits; }

    // the next pass: histogram, count scan, scatter
    pm_status step()
    {
        const int nb = bits - shift < 8 ? bits - shift : 8;
        const uint32_t mask = (1u << nb) - 1u;
        {
            ProfScope prof(n_hist.c_str(), s);
            hipLaunchKernelGGL(radix_histogram, dim3((unsigned)tiles), dim3(kRadixThreads), 0, s, ki, N, shift, mask,
                               counts, tiles);
            PM_HIP(hipGetLastError());
        }
        {
            ProfScope prof(n_scan.c_str(), s);
            hipLaunchKernelGGL(radix_chunk_sums, dim3((unsigned)chunks), dim3(kBlock), 0, s, counts, tiles, chunk);
            hipLaunchKernelGGL(radix_chunk_scan, dim3(1), dim3(kRadixParts * kBlock), 0, s, chunk, chunks);
            hipLaunchKernelGGL(radix_chunk_apply, dim3((unsigned)chunks), dim3(kBlock), 0, s, counts, chunk, tiles,
                               offs);
            PM_HIP(hipGetLastError());
        }
        {
            const bool last = shift + 8 >= bits;
            uint64_t *po = (last && pair_out) ? pair_out : nullptr;
            uint32_t *so = last ? sample_out : nullptr;
            ProfScope prof(n_scat.c_str(), s);
            uint32_t *kw = (po || (last && !keys_wanted)) ? nullptr : ko;
            hipLaunchKernelGGL(radix_scatter, dim3((unsigned)tiles), dim3(kRadixThreads), 0, s, ki, vi, N, shift, mask,
                               offs, tiles, kw, vo, po, so);
            PM_HIP(hipGetLastError());
        }
        out_k = ko;
        out_v = vo;
        ki = ko;
        vi = vo;
        ko = (ko == k0) ? k1 : k0;
        vo = (vo == v0) ? v1 : v0;
        shift += 8;
        if (done() && (pair_out || !keys_wanted)) out_k = nullptr;
        return PM_OK;
    }
};

inline pm_status radix_sort(const char *name, const uint32_t *in_k, const uint32_t *in_v, uint32_t *k0, uint32_t *v0,
                            uint32_t *k1, uint32_t *v1, int64_t N, int bits, void *scratch, hipStream_t s,
                            uint32_t **out_k, uint32_t **out_v, uint64_t *pair_out = nullptr,
                            uint32_t *sample_out = nullptr, bool keys_wanted = true)
{
    *out_k = k0;
    *out_v = v0;
    if (N <= 1 || bits <= 0) {
        // nothing to sort: copy the input through (values, pairs, samples)
        if (N > 0) {
            hipLaunchKernelGGL(radix_pair_copy, dim3(grid_for(N, kBlock, 1 << 22)), dim3(kBlock), 0, s, in_k, in_v, N,
                               pair_out, sample_out, v0);
            PM_HIP(hipGetLastError());
            if (!pair_out) PM_HIP(hipMemcpyAsync(k0, in_k, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, s));
        }
        if (pair_out) *out_k = nullptr;
        return PM_OK;
    }
    RadixRun r(name, in_k, in_v, k0, v0, k1, v1, N, bits, scratch, s, pair_out, sample_out, keys_wanted);
    while (!r.done()) PM_TRY(r.step());
    *out_k = r.out_k;
    *out_v = r.out_v;
    return PM_OK;
}

}  // namespace pm
