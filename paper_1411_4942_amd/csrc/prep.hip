// Graph preparation: validation, degrees, the degree-order relabel of
// Section 4, tau/lambda weights with their prefix sums (Sections 3 and 4),
// N_1 (Algorithm 2) and the guide tables of the edge draw.
//
// The relabelled rows are built already sorted, one size class of rows per
// launch (lane, wave and block sorts; global radix sorts for the few hub
// rows).  One stable sort of the finished slots by column then lists, at
// position q, the slot holding the reverse of slot q: that permutation is at
// once the symmetry check and the reverse slot map the lambda weights need.
// The weights are parked with per-tile sums, and a second pass turns them
// into both prefix sums and fills the guide tables.
#include "graph.hpp"
#include "profile.hpp"
#include "radix.hpp"
#include "rowhash.hpp"
#include "streams.hpp"

#include <algorithm>
#include <vector>

namespace pm {

enum : uint32_t {
    ERR_OFFSETS = 1u,
    ERR_RANGE = 2u,
    ERR_LOOP = 4u,
    ERR_ORDER = 8u,
    ERR_ASYM = 16u,
    ERR_OVF_TAU = 32u,
    ERR_OVF_LAM = 64u,
    ERR_GUIDE = 128u,  // guide write out of range: only from inconsistent weights
};

struct PrepStats {
    uint32_t err;
    uint32_t dmax;
    uint64_t isolated;
    uint64_t n1_lo;
    uint64_t n1_hi;
    uint32_t nlong_tau;
    uint32_t nlong_lam;
    U64x2 totals;        // (2W, 2 Lambda) as summed by the weights scan
    uint32_t shift_tau;  // guide bucket width 2^shift of each sampler
    uint32_t shift_lam;
    uint64_t nb_tau;     // guide buckets of each sampler
    uint64_t nb_lam;
};

// Guide shape: the smallest bucket width 2^shift with at most `target`
// buckets over [0, R) (target >= 2, so shift <= 63).  Same on host and device.
__host__ __device__ inline uint32_t guide_shift(uint64_t R, uint64_t target)
{
    uint32_t sh = 0;
    while (sh < 63 && ((R - 1) >> sh) + 1 > target) ++sh;
    return sh;
}

__host__ __device__ inline uint64_t guide_target(int64_t slots)
{
    return slots / 4 > 2 ? (uint64_t)(slots / 4) : 2ull;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_degrees(const int64_t *__restrict__ off, int64_t n, int64_t slots,
                                                    uint32_t *__restrict__ deg, PrepStats *st)
{
    uint32_t err = 0, dmax = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = off[v], b = off[v + 1];
        if (a < 0 || b < a || b > slots) {
            err |= ERR_OFFSETS;
            deg[v] = 0;
            continue;
        }
        uint32_t d = (uint32_t)(b - a);
        deg[v] = d;
        dmax = d > dmax ? d : dmax;
    }
    if (err) atomicOr(&st->err, err);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint32_t x = __shfl_xor(dmax, o, kWave);
        dmax = x > dmax ? x : dmax;
    }
    // one atomic per block: contention on st->dmax, not bandwidth, bounds this kernel
    __shared__ uint32_t s_max[kBlock / kWave];
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) m = s_max[i] > m ? s_max[i] : m;
        if (m) atomicMax(&st->dmax, m);
    }
}

__global__ void k_rank_from_order(const uint32_t *__restrict__ order, int32_t *__restrict__ rank, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rank[order[i]] = (int32_t)i;
}

struct DegIn {
    const uint32_t *d;
    __device__ __forceinline__ uint64_t operator()(int64_t i) const { return d[i]; }
};
struct OffOut {
    uint32_t *off;  // writes off[i+1] (below 2^32: the slot count is)
    __device__ __forceinline__ void operator()(int64_t i, uint64_t incl, uint64_t) const { off[i + 1] = (uint32_t)incl; }
};

// ---------------------------------------------------------------------------
// Relabelled rows built sorted (Section 4's order: ids are ranks, rows
// ascending).  New row i is input row u = order[i] with every column c
// mapped to rank[c]; rows are sorted where they are built, by size class:
//   degree <= 16          16 lanes per row, a sorting network across them
//   16 < degree <= 64     one wave per row, a sorting network across lanes
//   64 < degree <= 256    one wave per row, a sorting network on 2 (up to
//                         128) or 4 keys per lane
//   256 < degree <= 8192  one block per row sized to the class (64, 256 or
//                         512 threads), stable LSD radix sort with the keys
//                         in registers and one LDS exchange buffer (a third
//                         of the LDS of a two-buffer sort, so more blocks
//                         share a CU)
//   8192 < degree <= 16384  one block of 1024 per row, stable LSD radix sort
//                         between two LDS buffers
//   16384 < degree <= 32768  one block of 1024 per row, keys in registers
//                         and one LDS exchange buffer (128 KB)
//   degree > 32768        (the few hub rows, all at the end of the order)
//                         chunks of 32768 sorted as the class above, then
//                         merged within each row
// Each class writes col, edge = row | col << 32, and ladder level 1 (every
// 32nd column) at the row's final slots, and checks the input row (column
// range, self-loop, strictly ascending).
// ---------------------------------------------------------------------------

// the checks of one input slot p (row u, previous column prev or -1)
__device__ __forceinline__ uint32_t slot_checks(int64_t c, int64_t u, int64_t prev, int64_t n)
{
    uint32_t e = 0;
    if (c < 0 || c >= n) e |= ERR_RANGE;
    if (c == u) e |= ERR_LOOP;
    if (prev >= c) e |= ERR_ORDER;
    return e;
}

__device__ __forceinline__ void emit_slot(int64_t p, uint32_t row, uint32_t c, uint32_t *__restrict__ col,
                                          uint64_t *__restrict__ edge, uint32_t *__restrict__ ladder1)
{
    col[p] = c;
    edge[p] = (uint64_t)row | ((uint64_t)c << 32);
    if (ladder1 && (p & 31) == 0) ladder1[p >> 5] = c;
}

__device__ __forceinline__ void cswap(uint32_t &a, uint32_t &b)
{
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// rows [r0, r1) with degree <= W, a group of W lanes each (W = 16: four rows
// per wave; W = 64: one): slot j of a row is lane j of its group, so loads
// and stores coalesce; a bitonic network across the group's lanes (absent
// entries are 0xFFFFFFFF and sort last).  A slot's predecessor for the order
// check comes from the lane below.
template <int W>
__global__ __launch_bounds__(kBlock) void k_rows_group(const int64_t *__restrict__ off_in,
                                                       const int32_t *__restrict__ col_in,
                                                       const uint32_t *__restrict__ order,
                                                       const int32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ off_new, int64_t n, int64_t r0,
                                                       int64_t r1, uint32_t *__restrict__ col,
                                                       uint64_t *__restrict__ edge, uint32_t *__restrict__ ladder1,
                                                       PrepStats *st)
{
    static_assert(W == 16 || W == 64, "a quarter wave or a wave per row");
    const int64_t i = r0 + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / W;
    if (W == kWave && i >= r1) return;  // whole waves leave together
    const int j = lane_id() & (W - 1);
    const bool row = i < r1;  // W = 16: the last wave may hold fewer rows
    int64_t u = 0, a = 0, d = 0;
    if (row) {
        u = order[i];
        a = off_in[u];
        d = off_in[u + 1] - a;
    }
    const bool ok = row && j < d;
    const int32_t c = ok ? col_in[a + j] : 0;
    const int32_t below = __shfl_up(c, 1, W);  // every lane takes part
    uint32_t err = 0, v = 0xFFFFFFFFu;
    if (ok) {
        err = slot_checks(c, u, j > 0 ? (int64_t)below : -1, n);
        v = (c >= 0 && c < n) ? (uint32_t)rank[c] : 0u;
    }
#pragma unroll
    for (int size = 2; size <= W; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint32_t o = __shfl_xor(v, stride, W);
            const bool up = (j & size) == 0, low = (j & stride) == 0;
            v = (up == low) ? (v < o ? v : o) : (v < o ? o : v);
        }
    if (ok) emit_slot(off_new[i] + j, (uint32_t)i, v, col, edge, ladder1);
    if (err) atomicOr(&st->err, err);
}

// One compare step of a bitonic network on 64 * ITEMS keys held as element
// e = lane * ITEMS + j in k[j]: pairs (e, e ^ M), the lower element keeping
// the smaller key.  M below ITEMS pairs registers of one lane; otherwise
// lanes lane ^ (M / ITEMS) exchange register j ^ (M % ITEMS), and the lane
// whose bit for M's top bit is clear holds the lower element.  M is a
// compile-time constant after unrolling.
template <int ITEMS>
__device__ __forceinline__ void bitonic_step(uint32_t (&k)[ITEMS], int lane, int M)
{
    if (M < ITEMS) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
            if ((j ^ M) > j) cswap(k[j], k[j ^ M]);
    } else {
        const int ml = M / ITEMS, mj = M % ITEMS;
        const int top = 1 << (31 - __builtin_clz((unsigned)ml));
        const bool lower = (lane & top) == 0;
        uint32_t o[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) o[j] = __shfl_xor(k[j ^ mj], ml, kWave);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) k[j] = lower ? (k[j] < o[j] ? k[j] : o[j]) : (k[j] < o[j] ? o[j] : k[j]);
    }
}

// rows [r0, r1) with 64 < degree <= 64 * ITEMS, one wave each: bitonic
// sorting network on 64 * ITEMS keys in registers (absent entries are
// 0xFFFFFFFF and sort last), element e = lane * ITEMS + j so that the
// frequent short strides stay inside a lane.  Each merge stage of size 2^p
// opens with the mirror step (e against e ^ (2^p - 1)) and continues with
// half-cleaners (e against e ^ 2^q for q = p - 2 .. 0).
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_rows_bitonic(const int64_t *__restrict__ off_in,
                                                         const int32_t *__restrict__ col_in,
                                                         const uint32_t *__restrict__ order,
                                                         const int32_t *__restrict__ rank,
                                                         const uint32_t *__restrict__ off_new, int64_t n, int64_t r0,
                                                         int64_t r1, uint32_t *__restrict__ col,
                                                         uint64_t *__restrict__ edge, uint32_t *__restrict__ ladder1,
                                                         PrepStats *st)
{
    static_assert(ITEMS == 2 || ITEMS == 4, "two or four keys per lane");
    constexpr int LOG_N = ITEMS == 2 ? 7 : 8;
    const int64_t i = r0 + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (i >= r1) return;  // whole waves leave together
    const int lane = lane_id();
    const int64_t u = order[i], a = off_in[u];
    const int d = (int)(off_in[u + 1] - a);  // <= 64 * ITEMS by the class bounds
    int32_t c[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int e = lane * ITEMS + j;
        c[j] = e < d ? col_in[a + e] : 0;
    }
    const int32_t left = __shfl_up(c[ITEMS - 1], 1, kWave);  // element lane * ITEMS - 1
    uint32_t err = 0, k[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int e = lane * ITEMS + j;
        k[j] = 0xFFFFFFFFu;
        if (e < d) {
            const int64_t cv = c[j];
            const int64_t prev = j > 0 ? (int64_t)c[j - 1] : (lane > 0 ? (int64_t)left : -1);
            err |= slot_checks(cv, u, prev, n);
            k[j] = (cv >= 0 && cv < n) ? (uint32_t)rank[cv] : 0u;
        }
    }
#pragma unroll
    for (int p = 1; p <= LOG_N; ++p) {
        bitonic_step<ITEMS>(k, lane, (1 << p) - 1);
#pragma unroll
        for (int q = p - 2; q >= 0; --q) bitonic_step<ITEMS>(k, lane, 1 << q);
    }
    const int64_t dst = off_new[i];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const int e = lane * ITEMS + j;
        if (e < d) emit_slot(dst + e, (uint32_t)i, k[j], col, edge, ladder1);
    }
    if (err) atomicOr(&st->err, err);
}

// Stable LSD radix sort of up to THREADS * ITEMS keys in LDS (8-bit digits,
// `bits` key bits): wave w ranks its contiguous chunk with ballots and per-wave
// digit counters, the counters become output positions, the keys move to the
// other buffer.  Returns the buffer holding the result.  Every thread of the
// block calls it.
// Rank of a key with digit `dig` among the keys of its wave pass (stable:
// lanes below first), counted on top of the wave's running digit counts cnt.
__device__ __forceinline__ uint32_t wave_digit_rank(uint32_t dig, bool ok, uint64_t lt_mask, uint32_t *cnt)
{
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
        const uint64_t bal = __ballot((dig >> bb) & 1u);
        peers &= ((dig >> bb) & 1u) ? bal : ~bal;
    }
    const uint32_t below = __popcll(peers & lt_mask);
    const uint32_t base = cnt[dig];
    if (ok && below == 0) cnt[dig] = base + (uint32_t)__popcll(peers);
    return base + below;
}

// Per-wave digit counts s_cnt[w * 256 + d] to the first output position of
// wave w's keys with digit d (digits in order, waves in order within one).
template <int THREADS>
__device__ __forceinline__ void block_digit_offsets(uint32_t *s_cnt, uint32_t *s_tot)
{
    constexpr int W = THREADS / kWave;
    const int t = threadIdx.x, lane = lane_id();
    for (int d0 = t; d0 < 256; d0 += THREADS) {
        uint32_t tot = 0;
        for (int ww = 0; ww < W; ++ww) tot += s_cnt[ww * 256 + d0];
        s_tot[d0] = tot;
    }
    __syncthreads();
    if (t < kWave) {  // exclusive scan of the 256 totals, 4 per lane
        const uint32_t v0 = s_tot[4 * t], v1 = s_tot[4 * t + 1], v2 = s_tot[4 * t + 2], v3 = s_tot[4 * t + 3];
        const uint32_t loc = v0 + v1 + v2 + v3;
        uint32_t incl = loc;
#pragma unroll
        for (int dd = 1; dd < kWave; dd <<= 1) {
            const uint32_t o = __shfl_up(incl, dd, kWave);
            if (lane >= dd) incl += o;
        }
        const uint32_t ex = incl - loc;
        s_tot[4 * t] = ex;
        s_tot[4 * t + 1] = ex + v0;
        s_tot[4 * t + 2] = ex + v0 + v1;
        s_tot[4 * t + 3] = ex + v0 + v1 + v2;
    }
    __syncthreads();
    for (int d0 = t; d0 < 256; d0 += THREADS) {
        uint32_t run = s_tot[d0];
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t c = s_cnt[ww * 256 + d0];
            s_cnt[ww * 256 + d0] = run;
            run += c;
        }
    }
    __syncthreads();
}

// Keys per wave in the block sorts: the nk keys split into W contiguous runs
// of a whole number of wave rows, so every wave has work whatever nk is (a
// fixed ITEMS-row run per wave would idle the upper waves on rows near the
// lower bound of their size class).  Wave w ranks keys [w * per, (w + 1) *
// per) in order, item i of it being key w * per + i * kWave + lane; per <=
// ITEMS * kWave when nk <= THREADS * ITEMS.
template <int THREADS>
__device__ __forceinline__ int keys_per_wave(int nk)
{
    constexpr int W = THREADS / kWave;
    return (nk + W * kWave - 1) / (W * kWave) * kWave;
}

// Stable LSD radix sort (8-bit digits) of nk <= THREADS * ITEMS keys in LDS,
// ping-ponging between a and b; returns the buffer holding the result.
template <int THREADS, int ITEMS>
__device__ uint32_t *block_radix_lds(uint32_t *a, uint32_t *b, int nk, int bits, uint32_t *s_cnt, uint32_t *s_tot)
{
    constexpr int W = THREADS / kWave;
    const int t = threadIdx.x, w = t / kWave, lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int per = keys_per_wave<THREADS>(nk);
    for (int shift = 0; shift < bits; shift += 8) {
        const uint32_t mask = (bits - shift >= 8) ? 0xFFu : ((1u << (bits - shift)) - 1u);
        for (int j = t; j < W * 256; j += THREADS) s_cnt[j] = 0;
        __syncthreads();
        uint32_t rank[ITEMS], dig[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i * kWave >= per) break;  // wave-uniform
            const int idx = w * per + i * kWave + lane;
            const bool ok = idx < nk;
            dig[i] = ok ? (a[idx] >> shift) & mask : 0u;
            rank[i] = wave_digit_rank(dig[i], ok, lt_mask, s_cnt + w * 256);
        }
        __syncthreads();
        block_digit_offsets<THREADS>(s_cnt, s_tot);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i * kWave >= per) break;
            const int idx = w * per + i * kWave + lane;
            if (idx < nk) b[s_cnt[w * 256 + dig[i]] + rank[i]] = a[idx];
        }
        __syncthreads();
        uint32_t *tmp = a;
        a = b;
        b = tmp;
    }
    return a;
}

// The same sort with the keys held in registers between passes (key[i] is
// item i as above) and one LDS buffer for the exchange: twice the capacity in
// the same LDS.  Each key's rank among its wave's keys of the same digit is
// kept in a register from the counting step to the scatter.  buf holds
// THREADS * ITEMS words; the sorted keys end in its first nk (it must hold
// the input keys when bits == 0).
template <int THREADS, int ITEMS>
__device__ __forceinline__ void block_radix_reg(uint32_t (&key)[ITEMS], uint32_t *buf, int nk, int bits,
                                                uint32_t *s_cnt, uint32_t *s_tot)
{
    constexpr int W = THREADS / kWave;
    const int t = threadIdx.x, w = t / kWave, lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int per = keys_per_wave<THREADS>(nk);
    for (int shift = 0; shift < bits; shift += 8) {
        const uint32_t mask = (bits - shift >= 8) ? 0xFFu : ((1u << (bits - shift)) - 1u);
        for (int j = t; j < W * 256; j += THREADS) s_cnt[j] = 0;
        __syncthreads();
        uint32_t rank[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int idx = w * per + i * kWave + lane;
            const bool ok = idx < nk;
            // an opaque copy: the ballots of later items would otherwise be
            // computed ahead and held in registers
            uint32_t k = key[i];
            asm volatile("" : "+v"(k));
            // every item ranks (absent ones count nothing), so that each
            // register of rank is written on every path
            rank[i] = i * kWave < per ? wave_digit_rank(ok ? (k >> shift) & mask : 0u, ok, lt_mask, s_cnt + w * 256)
                                      : 0u;
        }
        __syncthreads();
        block_digit_offsets<THREADS>(s_cnt, s_tot);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int idx = w * per + i * kWave + lane;
            if (i * kWave < per && idx < nk) buf[s_cnt[w * 256 + ((key[i] >> shift) & mask)] + rank[i]] = key[i];
        }
        __syncthreads();
        if (shift + 8 >= bits) break;  // the result stays in buf
        // unconditional reads (every index is below THREADS * ITEMS): a
        // conditional write to one register of key would make the compiler
        // spill the whole array at every branch
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) key[i] = buf[w * per + i * kWave + lane];
        // buf is written again only after the next pass's first barrier
    }
}

// rows [r0, r0 + gridDim.x), degree <= THREADS * ITEMS, one block each
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_rows_block(const int64_t *__restrict__ off_in,
                                                        const int32_t *__restrict__ col_in,
                                                        const uint32_t *__restrict__ order,
                                                        const int32_t *__restrict__ rank,
                                                        const uint32_t *__restrict__ off_new, int64_t n, int64_t r0,
                                                        int bits, uint32_t *__restrict__ col,
                                                        uint64_t *__restrict__ edge, uint32_t *__restrict__ ladder1,
                                                        PrepStats *st)
{
    constexpr int CAP = THREADS * ITEMS;
    __shared__ uint32_t s_a[CAP], s_b[CAP];
    __shared__ uint32_t s_cnt[(THREADS / kWave) * 256];
    __shared__ uint32_t s_tot[256];
    const int64_t i = r0 + blockIdx.x;
    const int64_t u = order[i], a = off_in[u];
    const int d = (int)(off_in[u + 1] - a);  // <= CAP by the class bounds
    uint32_t err = 0;
    for (int j = threadIdx.x; j < d; j += THREADS) {
        const int64_t c = col_in[a + j];
        const int64_t prev = j > 0 ? (int64_t)col_in[a + j - 1] : -1;
        err |= slot_checks(c, u, prev, n);
        s_a[j] = (c >= 0 && c < n) ? (uint32_t)rank[c] : 0u;
    }
    __syncthreads();
    const uint32_t *sorted = block_radix_lds<THREADS, ITEMS>(s_a, s_b, d, bits, s_cnt, s_tot);
    const int64_t dst = off_new[i];
    for (int j = threadIdx.x; j < d; j += THREADS) emit_slot(dst + j, (uint32_t)i, sorted[j], col, edge, ladder1);
    if (err) atomicOr(&st->err, err);
}

// rows [r0, r0 + gridDim.x), degree <= THREADS * ITEMS, one block each,
// keys in registers (block_radix_reg); the row enters and leaves through
// the LDS buffer
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_rows_block_reg(const int64_t *__restrict__ off_in,
                                                            const int32_t *__restrict__ col_in,
                                                            const uint32_t *__restrict__ order,
                                                            const int32_t *__restrict__ rank,
                                                            const uint32_t *__restrict__ off_new, int64_t n,
                                                            int64_t r0, int bits, uint32_t *__restrict__ col,
                                                            uint64_t *__restrict__ edge,
                                                            uint32_t *__restrict__ ladder1, PrepStats *st)
{
    constexpr int CAP = THREADS * ITEMS;
    __shared__ uint32_t s_buf[CAP];
    __shared__ uint32_t s_cnt[(THREADS / kWave) * 256];
    __shared__ uint32_t s_tot[256];
    const int64_t i = r0 + blockIdx.x;
    const int64_t u = order[i], a = off_in[u];
    const int d = (int)(off_in[u + 1] - a);  // <= CAP by the class bounds
    const int w = threadIdx.x / kWave, lane = lane_id();
    uint32_t err = 0;
    for (int j = threadIdx.x; j < d; j += THREADS) {
        const int64_t c = col_in[a + j];
        const int64_t prev = j > 0 ? (int64_t)col_in[a + j - 1] : -1;
        err |= slot_checks(c, u, prev, n);
        s_buf[j] = (c >= 0 && c < n) ? (uint32_t)rank[c] : 0u;
    }
    __syncthreads();
    uint32_t key[ITEMS];
    // unconditional reads, as in block_radix_reg
    const int per = keys_per_wave<THREADS>(d);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) key[it] = s_buf[w * per + it * kWave + lane];
    // the first pass writes s_buf only after its own barriers
    block_radix_reg<THREADS, ITEMS>(key, s_buf, d, bits, s_cnt, s_tot);
    const int64_t dst = off_new[i];
    for (int j = threadIdx.x; j < d; j += THREADS) emit_slot(dst + j, (uint32_t)i, s_buf[j], col, edge, ladder1);
    if (err) atomicOr(&st->err, err);
}

// Hub rows [r0, n) (degree > 32768: a few rows of up to hundreds of
// thousands of slots).  Hub-local position q stands for slot off_new[r0] + q.
// Each row is cut into chunks of kHubChunk slots; one block sorts a chunk
// with the keys in registers (as the largest block class), then rounds of
// pairwise merges, the run length doubling each round, leave one sorted run
// per row, which the round that finishes it writes to the row's slots.
constexpr int kHubChunk = 32768;                // 1024 threads x 32 keys
constexpr int kMergeTile = 2048;                // merged slots per block and round
constexpr int kMergePer = kMergeTile / kBlock;  // per thread

// hstart[h] = off_new[r0 + h] - off_new[r0] for h in [0, H] (H = n - r0 hub
// rows) and cstart[h] = the chunks of hub rows before h (cstart[H] = all of
// them); one block
__global__ __launch_bounds__(kBlock) void k_hub_layout(const uint32_t *__restrict__ off_new, int64_t r0, int64_t H,
                                                       uint32_t *__restrict__ hstart, uint32_t *__restrict__ cstart)
{
    __shared__ uint32_t s_sum[kBlock];
    const int t = threadIdx.x;
    const int64_t per = (H + kBlock - 1) / kBlock;
    const int64_t h0 = t * per < H ? t * per : H, h1 = h0 + per < H ? h0 + per : H;
    const uint32_t p0 = off_new[r0];
    uint32_t local = 0;
    for (int64_t h = h0; h < h1; ++h)
        local += (off_new[r0 + h + 1] - off_new[r0 + h] + kHubChunk - 1) / kHubChunk;
    s_sum[t] = local;
    __syncthreads();
    if (t == 0) {  // exclusive scan of the 256 thread sums
        uint32_t run = 0;
        for (int i = 0; i < kBlock; ++i) {
            const uint32_t x = s_sum[i];
            s_sum[i] = run;
            run += x;
        }
    }
    __syncthreads();
    uint32_t run = s_sum[t];
    for (int64_t h = h0; h < h1; ++h) {
        hstart[h] = off_new[r0 + h] - p0;
        cstart[h] = run;
        run += (off_new[r0 + h + 1] - off_new[r0 + h] + kHubChunk - 1) / kHubChunk;
    }
    if (t == kBlock - 1) {  // the last thread's range ends at H
        hstart[H] = off_new[r0 + H] - p0;
        cstart[H] = run;
    }
}

// last h in [0, H) with start[h] <= x (start[0] = 0 <= x)
__device__ __forceinline__ int64_t hub_of(const uint32_t *__restrict__ start, int64_t H, uint64_t x)
{
    int64_t lo = 0, hi = H;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (start[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// chunk blockIdx.x of the hub rows sorted into out (hub-local positions);
// the grid is an upper bound on the chunk count, blocks beyond it leave
template <int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_hub_chunks(const int64_t *__restrict__ off_in,
                                                        const int32_t *__restrict__ col_in,
                                                        const uint32_t *__restrict__ order,
                                                        const int32_t *__restrict__ rank,
                                                        const uint32_t *__restrict__ hstart,
                                                        const uint32_t *__restrict__ cstart, int64_t n, int64_t r0,
                                                        int64_t H, int bits, uint32_t *__restrict__ out, PrepStats *st)
{
    constexpr int CAP = THREADS * ITEMS;
    static_assert(CAP == kHubChunk, "one chunk per block");
    __shared__ uint32_t s_buf[CAP];
    __shared__ uint32_t s_cnt[(THREADS / kWave) * 256];
    __shared__ uint32_t s_tot[256];
    const uint32_t b = blockIdx.x;
    if (b >= cstart[H]) return;  // the whole block
    const int64_t h = hub_of(cstart, H, b), i = r0 + h, u = order[i], a = off_in[u];
    const int64_t d = off_in[u + 1] - a, c0 = (int64_t)(b - cstart[h]) * CAP;
    const int nk = (int)(d - c0 < CAP ? d - c0 : CAP);
    const int w = threadIdx.x / kWave, lane = lane_id();
    uint32_t err = 0;
    for (int j = threadIdx.x; j < nk; j += THREADS) {
        const int64_t jj = c0 + j;
        const int64_t c = col_in[a + jj];
        const int64_t prev = jj > 0 ? (int64_t)col_in[a + jj - 1] : -1;  // across chunk edges too
        err |= slot_checks(c, u, prev, n);
        s_buf[j] = (c >= 0 && c < n) ? (uint32_t)rank[c] : 0u;
    }
    __syncthreads();
    uint32_t key[ITEMS];
    // unconditional reads, as in block_radix_reg; a hub row means n > 32768,
    // so bits >= 16 and the sort makes passes
    const int per = keys_per_wave<THREADS>(nk);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) key[it] = s_buf[w * per + it * kWave + lane];
    // the first pass writes s_buf only after its own barriers
    block_radix_reg<THREADS, ITEMS>(key, s_buf, nk, bits, s_cnt, s_tot);
    const int64_t q0 = hstart[h] + c0;
    for (int j = threadIdx.x; j < nk; j += THREADS) out[q0 + j] = s_buf[j];
    if (err) atomicOr(&st->err, err);
}

// One merge round over the hub rows still in several runs (degree > L; the
// hub rows ascend by degree, so they form a suffix).  In each such row the
// sorted runs [s, s + L) and [s + L, s + 2L) (s = the row's start plus a
// multiple of 2L, both cut at the row's end) become one sorted run; a run
// without a partner is carried over.  A row of degree <= 2L is finished by
// this round and goes straight to its final slots (col, edge, ladder);
// longer rows go to out for the next round.  Block b writes positions
// [qA + b kMergeTile, qA + (b + 1) kMergeTile) of [qA, T), qA the first
// active row's start, piece by piece where the tile crosses a pair's end:
// merge-path splits of the piece's first and last output, both inputs
// staged in LDS, kMergePer outputs per thread from its own split merged
// into LDS, then written out coalesced.  Ties
// take the first run (rows hold distinct keys unless the input fails its
// checks).  The grid covers [0, T); blocks past the end leave.
__global__ __launch_bounds__(kBlock) void k_hub_merge(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                      int64_t T, const uint32_t *__restrict__ hstart, int64_t H,
                                                      int64_t L, int64_t r0, int64_t p0, uint32_t *__restrict__ col,
                                                      uint64_t *__restrict__ edge, uint32_t *__restrict__ ladder1)
{
    __shared__ uint32_t s_a[kMergeTile], s_b[kMergeTile], s_out[kMergeTile];
    __shared__ int64_t s_split[2];
    const int t = threadIdx.x;
    // the first hub row of degree > L (H when none)
    int64_t lo0 = 0, hi0 = H;
    while (lo0 < hi0) {
        const int64_t mid = (lo0 + hi0) >> 1;
        if ((int64_t)(hstart[mid + 1] - hstart[mid]) > L)
            hi0 = mid;
        else
            lo0 = mid + 1;
    }
    int64_t q = (int64_t)hstart[lo0] + (int64_t)blockIdx.x * kMergeTile;
    if (q >= T) return;  // the whole block
    const int64_t tile_end = q + kMergeTile < T ? q + kMergeTile : T;
    while (q < tile_end) {  // block-uniform
        const int64_t h = hub_of(hstart, H, (uint64_t)q);
        const int64_t rs = hstart[h], re = hstart[h + 1];
        const int64_t ps = rs + (q - rs) / (2 * L) * (2 * L);
        const int64_t am = ps + L < re ? ps + L : re, pe = ps + 2 * L < re ? ps + 2 * L : re;
        const int64_t la = am - ps, lb = pe - am;
        const int64_t seg_end = tile_end < pe ? tile_end : pe;  // > q: ps <= q < pe
        const bool last = re - rs <= 2 * L;
        const uint32_t *A = in + ps, *B = in + am;
        if (t < 2) {
            // outputs [0, k) of the pair take A[0, i) and B[0, k - i): the
            // first i with A[i] > B[k - 1 - i]
            const int64_t k = (t ? seg_end : q) - ps;
            int64_t lo = k - lb > 0 ? k - lb : 0, hi = k < la ? k : la;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (A[mid] <= B[k - 1 - mid])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            s_split[t] = lo;
        }
        __syncthreads();
        const int64_t i0 = s_split[0], i1 = s_split[1];
        const int64_t j0 = (q - ps) - i0, j1 = (seg_end - ps) - i1;
        const int na = (int)(i1 - i0), nb = (int)(j1 - j0);  // na + nb = seg_end - q <= kMergeTile
        for (int x = t; x < na; x += kBlock) s_a[x] = A[i0 + x];
        for (int x = t; x < nb; x += kBlock) s_b[x] = B[j0 + x];
        __syncthreads();
        const int o0 = t * kMergePer, n_out = na + nb;
        if (o0 < n_out) {
            int lo = o0 - nb > 0 ? o0 - nb : 0, hi = o0 < na ? o0 : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_a[mid] <= s_b[o0 - 1 - mid])
                    lo = mid + 1;
                else
                    hi = mid;
            }
            int ia = lo, ib = o0 - lo;
            const int o1 = o0 + kMergePer < n_out ? o0 + kMergePer : n_out;
            for (int o = o0; o < o1; ++o) {
                const bool take_a = ib >= nb || (ia < na && s_a[ia] <= s_b[ib]);
                s_out[o] = take_a ? s_a[ia++] : s_b[ib++];
            }
        }
        __syncthreads();
        for (int o = t; o < n_out; o += kBlock) {
            if (last)
                emit_slot(p0 + q + o, (uint32_t)(r0 + h), s_out[o], col, edge, ladder1);
            else
                out[q + o] = s_out[o];
        }
        __syncthreads();  // s_a, s_b, s_out and s_split are refilled for the next piece
        q = seg_end;
    }
}

// first row of each size class (degrees ascend along the new order): cls[c]
// = first row with degree > {0, 16, 64, 128, 256, 1024, 4096, 8192, 16384,
// 32768}[c]; cls[10] = the first slot of row cls[9]
constexpr int kRowClasses = 10;
__global__ void k_row_classes(const uint32_t *__restrict__ deg, const uint32_t *__restrict__ off, int64_t n,
                              int64_t *cls)
{
    const uint32_t bound[kRowClasses] = {0u, 16u, 64u, 128u, 256u, 1024u, 4096u, 8192u, 16384u, 32768u};
    const int c = threadIdx.x;
    if (c >= kRowClasses) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {  // first row with deg > bound[c]
        const int64_t mid = (lo + hi) >> 1;
        if (deg[mid] > bound[c])
            hi = mid;
        else
            lo = mid + 1;
    }
    cls[c] = lo;
    cls[kRowClasses + 1 + c] = off[lo];  // first slot of the class's rows
    if (c == kRowClasses - 1) cls[kRowClasses] = off[lo];
}

// ladder level l from level l-1: next[i] = prev[32 i]
__global__ void k_ladder_level(const uint32_t *__restrict__ prev, int64_t count, uint32_t *__restrict__ next)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        next[i] = prev[i * 32];
}

__global__ void k_copy_u32(const uint32_t *__restrict__ a, uint32_t *__restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// Weights of a slot s = (u, v) with reverse slot r (Sections 3 and 4):
//   tau_s    = (d_u - 1)(d_v - 1)
//   lambda_s = L_{u,v} L_{v,u},  L_{u,v} = d_u - 1 - (position of v in row u)
// counts the neighbours of u after v; r's position in row v gives L_{v,u}.
// Symmetry is checked on the way: listing the slots by (col, row) must list
// the rows in the order of the slots' own rows (half 1: the reverse slot of s
// has column u, so in-degree = out-degree everywhere), and r must lie in row
// v (half 2).
//
// Launch 1 of the weights scan, written out for memory-level parallelism:
// both weights of every slot and their inclusive prefix sums inside the
// slot's segment of kPrefixSeg slots (one wave: kWItems rows of 64), and one
// pair of sums per segment.  Each thread issues the loads of kWBatch items
// before any store, so their gathers overlap; each row is one wave scan on
// top of the running sum of the rows before it.
constexpr int kWItems = 16;
constexpr int kWBatch = 16;
static_assert((int64_t)kWave * kWItems == kPrefixSeg, "one wave per prefix segment");

__global__ __launch_bounds__(kBlock) void k_weights_reduce(const uint64_t *__restrict__ edge,
                                                           const uint32_t *__restrict__ rev,
                                                           const uint32_t *__restrict__ off, int64_t N,
                                                           uint64_t *__restrict__ p_tau,
                                                           uint64_t *__restrict__ p_lam,
                                                           SlotRec *__restrict__ rec, U64x2 *__restrict__ seg_sums,
                                                           PrepStats *st)
{
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t seg = (int64_t)blockIdx.x * (kBlock / kWave) + w;
    const int64_t wave_base = seg * kPrefixSeg;
    if (wave_base >= N) return;  // wave-uniform; no barrier below
    uint32_t err = 0;
    U64x2 carry{0, 0};
#pragma unroll
    for (int h = 0; h < kWItems; h += kWBatch) {
        uint64_t e[kWBatch];
        uint32_t r[kWBatch];
#pragma unroll
        for (int i = 0; i < kWBatch; ++i) {
            const int64_t idx = wave_base + (int64_t)(h + i) * kWave + lane;
            const bool ok = idx < N;
            // read once here: keep them out of the cache the gathers use
            e[i] = ok ? __builtin_nontemporal_load(edge + idx) : 0ull;
            r[i] = ok ? __builtin_nontemporal_load(rev + idx) : 0u;
        }
        uint32_t ou[kWBatch], ou1[kWBatch], ov[kWBatch], ov1[kWBatch];
#pragma unroll
        for (int i = 0; i < kWBatch; ++i) {
            const uint32_t u = (uint32_t)e[i], v = (uint32_t)(e[i] >> 32);
            ou[i] = off[u];
            ou1[i] = off[u + 1];
            ov[i] = off[v];
            ov1[i] = off[v + 1];
        }
#pragma unroll
        for (int i = 0; i < kWBatch; ++i) {
            const int64_t idx = wave_base + (int64_t)(h + i) * kWave + lane;
            uint64_t tau = 0, lam = 0;
            if (idx < N) {
                const int64_t rr = r[i];
                // symmetry: slot rev[i] (the i-th slot ordered by column) lies
                // in row v.  Over all slots that makes every in-degree equal
                // its out-degree (rev is a bijection), so the slots of column
                // u fill exactly row u's positions, and slot rev[i] of row v
                // has column u: it is the reverse (v, u) of slot i.
                if (rr < (int64_t)ov[i] || rr >= (int64_t)ov1[i]) err |= ERR_ASYM;
                const int64_t du = (int64_t)ou1[i] - ou[i], dv = (int64_t)ov1[i] - ov[i];
                tau = (uint64_t)(du - 1) * (uint64_t)(dv - 1);
                const uint64_t luv = (uint64_t)(du - 1 - (idx - (int64_t)ou[i]));
                const uint64_t lvu = (uint64_t)(dv - 1 - (rr - (int64_t)ov[i]));
                lam = luv * lvu;
            }
            const U64x2 incl = wave_inclusive(U64x2{tau, lam}, PairSumOp(), U64x2{0, 0});
            if (idx < N) {
                // the slot's sampler record: column, its row bounds, row
                const uint32_t u = (uint32_t)e[i], v = (uint32_t)(e[i] >> 32);
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                const u32x4 r4 = {v, ov[i], ov1[i] - ov[i], u};
                __builtin_nontemporal_store(r4, reinterpret_cast<u32x4 *>(rec) + idx);
                // whole 512-byte rows per instruction, read again only by the
                // guide pass and the samplers: stream them past the cache
                __builtin_nontemporal_store(carry.a + incl.a, p_tau + idx);
                __builtin_nontemporal_store(carry.b + incl.b, p_lam + idx);
            }
            carry = PairSumOp()(carry, shfl_idx_t(incl, kWave - 1));
        }
    }
    if (err) atomicOr(&st->err, err);
    if (lane == 0) seg_sums[seg] = carry;
}

// exclusive prefixes of the segment sums, the totals after the last one
struct SegIn {
    const U64x2 *sums;
    __device__ __forceinline__ U64x2 operator()(int64_t i) const { return sums[i]; }
};
struct SegOut {
    uint64_t *seg_tau, *seg_lam;
    int64_t nseg;
    U64x2 *totals;
    __device__ __forceinline__ void operator()(int64_t i, U64x2 incl, U64x2 x) const
    {
        seg_tau[i] = incl.a - x.a;
        seg_lam[i] = incl.b - x.b;
        if (i == nseg - 1) {
            seg_tau[nseg] = incl.a;
            seg_lam[nseg] = incl.b;
            *totals = incl;
        }
    }
};

// Guide entries of slot i: the buckets whose start j << shift lies in
// [P[i-1], P[i]) point at slot i.  Runs longer than 64 buckets go to a list
// that k_guide_long fills with whole blocks.
// These writes run before the validation verdicts reach the host, so they
// are bounded by the guide and list sizes whatever the weights hold (with a
// valid graph every bucket index is below nb and the long list fits).
__device__ __forceinline__ void guide_fill(uint64_t prev, uint64_t cur, uint32_t shift, uint64_t nb, uint32_t slot,
                                           uint32_t *__restrict__ guide, uint32_t *__restrict__ long_list,
                                           uint32_t cap, uint32_t *nlong, uint32_t *err)
{
    if (cur <= prev) return;
    const uint64_t mask = (shift == 0) ? 0ull : ((1ull << shift) - 1ull);
    const uint64_t j0 = (prev >> shift) + ((prev & mask) != 0 ? 1u : 0u);
    const uint64_t j1 = (cur - 1) >> shift;
    if (j1 < j0) return;
    if (j1 >= nb) {
        atomicOr(err, (uint32_t)ERR_GUIDE);
        return;
    }
    if (j1 - j0 < 64) {
        for (uint64_t j = j0; j <= j1; ++j) guide[j] = slot;
    } else {
        const uint32_t idx = atomicAdd(nlong, 1u);
        if (idx < cap)
            long_list[idx] = slot;
        else
            atomicOr(err, (uint32_t)ERR_GUIDE);
    }
}


// guide shape from the totals, and the sentinel guide[nb] = last slot
__global__ void k_guide_setup(PrepStats *st, int64_t slots, uint32_t *guide_tau, uint32_t *guide_lam)
{
    const uint64_t target = guide_target(slots);
    const uint64_t Rt = st->totals.a, Rl = st->totals.b;
    const uint32_t sht = Rt ? guide_shift(Rt, target) : 0u, shl = Rl ? guide_shift(Rl, target) : 0u;
    const uint64_t nbt = Rt ? ((Rt - 1) >> sht) + 1 : 0, nbl = Rl ? ((Rl - 1) >> shl) + 1 : 0;
    st->shift_tau = sht;
    st->shift_lam = shl;
    st->nb_tau = nbt;  // <= target, the allocated size less the sentinel
    st->nb_lam = nbl;
    if (Rt) guide_tau[nbt] = (uint32_t)(slots - 1);
    if (Rl) guide_lam[nbl] = (uint32_t)(slots - 1);
}

// Launch 3 of the weights scan: the guide entries from the global prefixes
// (segment prefix + offset), and the wrap checks.  Each wave covers kWRounds
// rounds of kWave * kWV consecutive slots; in a round lane l owns kWV
// consecutive slots (16-byte loads covering whole lines per instruction).
// All rounds are loaded first; the prefix before a lane's first slot comes
// from the lane before it (lane 0: the previous round's last lane, or memory
// at the wave's first slot).
constexpr int kWV = 4;
constexpr int kWRounds = kWItems / kWV;

__device__ __forceinline__ uint64_t global_prefix(const uint64_t *__restrict__ P, const uint64_t *__restrict__ seg,
                                                  int64_t i)
{
    return P[i] + seg[i >> kPrefixSegShift];
}

__global__ __launch_bounds__(kBlock) void k_guide_fill(const uint64_t *__restrict__ p_tau,
                                                       const uint64_t *__restrict__ p_lam,
                                                       const uint64_t *__restrict__ seg_tau,
                                                       const uint64_t *__restrict__ seg_lam, int64_t N,
                                                       uint32_t *__restrict__ guide_tau,
                                                       uint32_t *__restrict__ guide_lam,
                                                       uint32_t *__restrict__ long_tau,
                                                       uint32_t *__restrict__ long_lam, uint32_t long_cap,
                                                       PrepStats *st)
{
    // an asymmetric input (found by the weights kernel) leaves the weights
    // inconsistent, so their bucket ranges could overlap without bound; the
    // build fails anyway, so the guide is not filled
    if (st->err & ERR_ASYM) return;
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t wave_base = (int64_t)blockIdx.x * (kBlock * kWItems) + (int64_t)w * (kWave * kWItems);
    const uint32_t sh_t = st->shift_tau, sh_l = st->shift_lam;
    const uint64_t nb_t = st->nb_tau, nb_l = st->nb_lam;
    uint32_t err = 0;
    uint64_t A[kWRounds][kWV], B[kWRounds][kWV];
#pragma unroll
    for (int rd = 0; rd < kWRounds; ++rd) {
        const int64_t s0 = wave_base + (int64_t)rd * (kWave * kWV) + (int64_t)lane * kWV;
        if (s0 + kWV <= N) {
            const uint4 *pa = reinterpret_cast<const uint4 *>(p_tau + s0);
            const uint4 *pb = reinterpret_cast<const uint4 *>(p_lam + s0);
            const uint4 x0 = pa[0], x1 = pa[1], y0 = pb[0], y1 = pb[1];
            const uint64_t ot = seg_tau[s0 >> kPrefixSegShift], ol = seg_lam[s0 >> kPrefixSegShift];
            A[rd][0] = ((uint64_t)x0.x | ((uint64_t)x0.y << 32)) + ot;
            A[rd][1] = ((uint64_t)x0.z | ((uint64_t)x0.w << 32)) + ot;
            A[rd][2] = ((uint64_t)x1.x | ((uint64_t)x1.y << 32)) + ot;
            A[rd][3] = ((uint64_t)x1.z | ((uint64_t)x1.w << 32)) + ot;
            B[rd][0] = ((uint64_t)y0.x | ((uint64_t)y0.y << 32)) + ol;
            B[rd][1] = ((uint64_t)y0.z | ((uint64_t)y0.w << 32)) + ol;
            B[rd][2] = ((uint64_t)y1.x | ((uint64_t)y1.y << 32)) + ol;
            B[rd][3] = ((uint64_t)y1.z | ((uint64_t)y1.w << 32)) + ol;
        } else {
#pragma unroll
            for (int j = 0; j < kWV; ++j) {
                A[rd][j] = s0 + j < N ? global_prefix(p_tau, seg_tau, s0 + j) : 0ull;
                B[rd][j] = s0 + j < N ? global_prefix(p_lam, seg_lam, s0 + j) : 0ull;
            }
        }
    }
    uint64_t carry_a = 0, carry_b = 0;  // the prefix before the round's first slot
    if (wave_base > 0 && wave_base <= N) {
        carry_a = global_prefix(p_tau, seg_tau, wave_base - 1);
        carry_b = global_prefix(p_lam, seg_lam, wave_base - 1);
    }
#pragma unroll
    for (int rd = 0; rd < kWRounds; ++rd) {
        const int64_t s0 = wave_base + (int64_t)rd * (kWave * kWV) + (int64_t)lane * kWV;
        const uint64_t up_a = __shfl_up(A[rd][kWV - 1], 1, kWave), up_b = __shfl_up(B[rd][kWV - 1], 1, kWave);
        uint64_t prev_a = lane ? up_a : carry_a, prev_b = lane ? up_b : carry_b;
        carry_a = __shfl(A[rd][kWV - 1], kWave - 1, kWave);
        carry_b = __shfl(B[rd][kWV - 1], kWave - 1, kWave);
#pragma unroll
        for (int j = 0; j < kWV; ++j) {
            const int64_t idx = s0 + j;
            if (idx < N) {
                // the running sum passed 2^64 exactly where it decreases
                if (A[rd][j] < prev_a) err |= ERR_OVF_TAU;
                if (B[rd][j] < prev_b) err |= ERR_OVF_LAM;
                guide_fill(prev_a, A[rd][j], sh_t, nb_t, (uint32_t)idx, guide_tau, long_tau, long_cap, &st->nlong_tau,
                           &st->err);
                guide_fill(prev_b, B[rd][j], sh_l, nb_l, (uint32_t)idx, guide_lam, long_lam, long_cap,
                           &st->nlong_lam, &st->err);
            }
            prev_a = A[rd][j];
            prev_b = B[rd][j];
        }
    }
    if (err) atomicOr(&st->err, err);
}

// N_1 = sum_v C(d_v, 3) in 128 bits; isolated vertices.  One pair of
// atomics per block.
__global__ __launch_bounds__(kBlock) void k_n1(const uint32_t *__restrict__ deg, int64_t n, PrepStats *st)
{
    __shared__ uint64_t s_lo[kBlock / kWave], s_hi[kBlock / kWave], s_iso[kBlock / kWave];
    unsigned __int128 acc = 0;
    uint64_t iso = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        uint64_t d = deg[v];
        iso += d == 0;
        if (d >= 3) {
            // C(d,3) = d (d-1) (d-2) / 6: divide the factors first, exactly
            uint64_t a = d, b = d - 1, c = d - 2;
            if (a % 3 == 0) a /= 3; else if (b % 3 == 0) b /= 3; else c /= 3;
            if ((a & 1) == 0) a >>= 1; else if ((b & 1) == 0) b >>= 1; else c >>= 1;
            acc += (unsigned __int128)(a * b) * c;
        }
    }
    uint64_t lo = (uint64_t)acc, hi = (uint64_t)(acc >> 64);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint64_t olo = __shfl_xor(lo, o, kWave), ohi = __shfl_xor(hi, o, kWave);
        uint64_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1u : 0u);
        lo = nlo;
        iso += __shfl_xor(iso, o, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_iso[w] = iso;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        lo = s_lo[0];
        hi = s_hi[0];
        iso = s_iso[0];
        for (int i = 1; i < kBlock / kWave; ++i) {
            uint64_t nlo = lo + s_lo[i];
            hi += s_hi[i] + (nlo < lo ? 1u : 0u);
            lo = nlo;
            iso += s_iso[i];
        }
        unsigned long long old = atomicAdd((unsigned long long *)&st->n1_lo, (unsigned long long)lo);
        uint64_t carry = (old + lo < old) ? 1u : 0u;
        atomicAdd((unsigned long long *)&st->n1_hi, (unsigned long long)(hi + carry));
        atomicAdd((unsigned long long *)&st->isolated, (unsigned long long)iso);
    }
}

__global__ __launch_bounds__(kBlock) void k_guide_long(const uint64_t *__restrict__ P,
                                                       const uint64_t *__restrict__ seg, const uint32_t *shift_p,
                                                       uint32_t *__restrict__ guide,
                                                       const uint32_t *__restrict__ long_list,
                                                       const uint32_t *nlong, uint32_t cap, const uint32_t *err)
{
    if (*err & (ERR_ASYM | ERR_GUIDE)) return;  // inconsistent weights: the build fails
    const uint32_t shift = *shift_p;
    const uint64_t mask = (shift == 0) ? 0ull : ((1ull << shift) - 1ull);
    const uint32_t cnt = *nlong < cap ? *nlong : cap;  // listed runs were checked against nb
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        uint32_t s = long_list[e];
        uint64_t prev = s > 0 ? global_prefix(P, seg, s - 1) : 0ull, cur = global_prefix(P, seg, s);
        uint64_t j0 = (prev >> shift) + ((prev & mask) != 0 ? 1u : 0u);
        uint64_t j1 = (cur - 1) >> shift;
        for (uint64_t j = j0 + threadIdx.x; j <= j1; j += blockDim.x) guide[j] = s;
    }
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------

namespace {


int grid_stream(int64_t n) { return grid_for(n, kBlock, 1 << 22); }

const char *err_text(uint32_t e)
{
    if (e & ERR_OFFSETS) return "row offsets decrease or leave [0, 2m]";
    if (e & ERR_RANGE) return "a column is not a vertex id";
    if (e & ERR_LOOP) return "self-loop";
    if (e & ERR_ORDER) return "a row is not strictly ascending (unsorted or repeated edge)";
    if (e & ERR_ASYM) return "adjacency is not symmetric (graph must be undirected)";
    return "invalid graph";
}

}  // namespace

void graph_free(pm_graph *g, hipStream_t s)
{
    if (!g) return;
    void *const arrays[] = {g->off,     g->col,     g->rec,       g->hash,      g->ladder,    g->deg,       g->rank,
                            g->p_tau,   g->p_lam,   g->seg_tau,   g->seg_lam,   g->guide_tau, g->guide_lam,
                            g->alias_tau, g->alias_lam};
    dev_free_batch(arrays, sizeof(arrays) / sizeof(arrays[0]), s);
    delete g;
}

// The row hash (rowhash.hip): `parts` is kRowHashSmall, kRowHashWide or both.
pm_status build_rowhash(const pm_graph *g, const int64_t rows[5], const int64_t slot_at[5], uint32_t *H,
                        hipStream_t s, int parts);

// Device bytes a prepared graph of n vertices and `slots` directed slots
// holds (what graph_create adds up in pm_graph::bytes).
uint64_t graph_bytes_for(int64_t n, int64_t slots)
{
    const uint64_t nn = (uint64_t)std::max<int64_t>(n, 1), ss = (uint64_t)std::max<int64_t>(slots, 1);
    uint64_t b = 4 * nn + 4 * nn + 4 * ((uint64_t)n + 1);
    const int top = ladder_top_for(slots);
    uint64_t total = 0;
    for (int l = 1; l <= top; ++l) total += (ladder_count(slots, l) + 31) / 32 * 32;
    if (top > 0) b += 4 * (total + 32);
    b += 20 * ss + 16 * ss;  // col and slot records; both prefix arrays
    b += 4 * (2 * ss + (uint64_t)kHashPad);  // row hash
    b += 2 * 8 * ((uint64_t)prefix_segments(slots) + 1);
    b += 2 * 4 * (guide_target(slots) + 1);
    return b;
}

pm_status graph_create(const pm_csr_view *csr, uint32_t flags, hipStream_t s, pm_graph **out)
{
    (void)flags;  // every check always runs: later kernels rely on them
    if (!csr || !out || !csr->row_offsets) {
        set_error("null argument");
        return PM_EINVAL;
    }
    *out = nullptr;
    const int64_t n = csr->n;
    if (n < 0 || n > (int64_t)INT32_MAX) {
        set_error("n must lie in [0, 2^31)");
        return PM_EINVAL;
    }
    ProfScope prof_total("prep_total", s);
    Temps tmp(s);

    // offsets bounds from the host side
    int64_t first = 0, slots = 0;
    if (csr->on_device) {
        PM_HIP(hipMemcpyAsync(&first, csr->row_offsets, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        PM_HIP(hipMemcpyAsync(&slots, csr->row_offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
    } else {
        first = csr->row_offsets[0];
        slots = csr->row_offsets[n];
    }
    if (first != 0 || slots < 0) {
        set_error(err_text(ERR_OFFSETS));
        return PM_EGRAPH;
    }
    if (slots >= (int64_t)UINT32_MAX) {
        set_error("2m must be below 2^32");
        return PM_EINVAL;
    }
    if (slots > 0 && !csr->cols) {
        set_error("null cols");
        return PM_EINVAL;
    }

    const int64_t *off_in = csr->row_offsets;
    const int32_t *col_in = csr->cols;
    if (!csr->on_device) {
        int64_t *o = nullptr;
        int32_t *c = nullptr;
        PM_TRY(tmp.get(&o, (size_t)n + 1));
        PM_TRY(tmp.get(&c, (size_t)std::max<int64_t>(slots, 1)));
        PM_HIP(hipMemcpyAsync(o, csr->row_offsets, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
        if (slots > 0) PM_HIP(hipMemcpyAsync(c, csr->cols, sizeof(int32_t) * slots, hipMemcpyHostToDevice, s));
        off_in = o;
        col_in = c;
    }

    pm_graph *g = new (std::nothrow) pm_graph();
    if (!g) return PM_ENOMEM;
    struct Guard {
        pm_graph *g;
        hipStream_t s;
        ~Guard()
        {
            if (g) graph_free(g, s);
        }
    } guard{g, s};
    PM_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->slots = slots;

    PrepStats *st = nullptr;
    PM_TRY(tmp.get(&st, 1));
    PM_TRY(fill_async<uint32_t>((uint32_t *)st, 0u, sizeof(PrepStats) / 4, s));
    PrepStats hst;

    const int64_t nn = std::max<int64_t>(n, 1), ss = std::max<int64_t>(slots, 1);
    uint32_t *deg_in = nullptr;
    PM_TRY(tmp.get(&deg_in, nn));
    if (n > 0) {
        ProfScope prof("degrees", s);
        hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, off_in, n, slots, deg_in, st);
        PM_HIP(hipGetLastError());
    }
    // the row walk below trusts the offsets: read the verdict first
    PM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (hst.err) {
        set_error(err_text(hst.err));
        return PM_EGRAPH;
    }
    g->dmax = hst.dmax;

    // vertex order: stable sort of ids by degree
    char *rscr = nullptr;
    PM_TRY(tmp.get(&rscr, radix_scratch_bytes(std::max<int64_t>(slots, n))));
    uint32_t *vk0, *vv0, *vk1, *vv1;
    PM_TRY(tmp.get(&vk0, nn));
    PM_TRY(tmp.get(&vv0, nn));
    PM_TRY(tmp.get(&vk1, nn));
    PM_TRY(tmp.get(&vv1, nn));
    uint32_t *sorted_deg, *order;
    PM_TRY(radix_sort("vertex_sort", deg_in, nullptr, vk0, vv0, vk1, vv1, n, bits_for((uint64_t)g->dmax), rscr, s,
                      &sorted_deg, &order));

    PM_TRY(dev_alloc((void **)&g->rank, sizeof(int32_t) * nn, s));
    PM_TRY(dev_alloc((void **)&g->deg, sizeof(uint32_t) * nn, s));
    PM_TRY(dev_alloc((void **)&g->off, sizeof(uint32_t) * (n + 1), s));
    g->bytes += sizeof(int32_t) * nn + sizeof(uint32_t) * nn + sizeof(uint32_t) * (n + 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_rank_from_order, dim3(grid_stream(n)), dim3(kBlock), 0, s, order, g->rank, n);
        hipLaunchKernelGGL(k_copy_u32, dim3(grid_stream(n)), dim3(kBlock), 0, s, sorted_deg, g->deg, n);
        PM_HIP(hipGetLastError());
    }
    PM_TRY(fill_async<uint32_t>(g->off, 0u, 1, s));
    {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<uint64_t>::bytes_for(n, 16)));
        PM_TRY((scan_launch<uint64_t, 16>(DegIn{g->deg}, OffOut{g->off}, n, SumOp<uint64_t>(), 0ull, scr, s)));
    }
    const int vbits = bits_for(n > 0 ? (uint64_t)(n - 1) : 0);
    // the column array is padded to whole 128-byte lines (ladder level 0)
    const int64_t ssp = (ss + 31) / 32 * 32 + 32;
    PM_TRY(dev_alloc((void **)&g->col, sizeof(uint32_t) * ssp, s));
    // (row, column) of every slot for the weights pass; the samplers read
    // the slot records it writes
    uint64_t *edge = nullptr;
    PM_TRY(tmp.get(&edge, (size_t)ss));
    PM_TRY(dev_alloc((void **)&g->rec, sizeof(SlotRec) * ss, s));
    g->bytes += (sizeof(uint32_t) + sizeof(SlotRec)) * ss;

    // ladder levels 1..top, count(l) = ceil(slots / 32^l); top is the smallest
    // level whose single line covers every slot (32^(top+1) >= slots)
    {
        uint64_t total = 0;
        const int top = ladder_top_for(slots);
        g->ladder_top = top;
        for (int l = 1; l <= top; ++l) {
            const uint64_t cnt = ladder_count(slots, l);
            g->ladder_off[l] = total;
            total += (cnt + 31) / 32 * 32;
        }
        if (top > 0) {
            PM_TRY(dev_alloc((void **)&g->ladder, sizeof(uint32_t) * (total + 32), s));
            g->bytes += sizeof(uint32_t) * (total + 32);
        }
    }
    uint32_t *ladder1 = g->ladder_top > 0 ? g->ladder + g->ladder_off[1] : nullptr;

    // the rows, sorted where they are built (by size class)
    int64_t cls[2 * kRowClasses + 1] = {0};  // first row of each class, then the hub rows' and classes' first slots
    if (slots > 0) {
        int64_t *cls_d = nullptr;
        PM_TRY(tmp.get(&cls_d, 2 * kRowClasses + 1));
        hipLaunchKernelGGL(k_row_classes, dim3(1), dim3(kWave), 0, s, g->deg, g->off, n, cls_d);
        PM_HIP(hipGetLastError());
        PM_HIP(hipMemcpyAsync(cls, cls_d, sizeof(cls), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        ProfScope prof("build_rows", s);
        // the rows above 8192 (one block of 1024 per row or chunk, whose few
        // large blocks leave CUs idle at the ends of their launches) run on two
        // side streams, forked from s before the other classes are enqueued
        // (they read only the offsets, order and rank) and joined back; the
        // many small blocks of the other classes fill the CUs beside them
        const int64_t T = slots - cls[kRowClasses];
        const int64_t rt = cls[kRowClasses - 1], H = n - rt;
        uint32_t *run0 = nullptr, *run1 = nullptr, *hstart = nullptr, *cstart = nullptr;
        if (T > 0) {
            PM_TRY(tmp.get(&run0, (size_t)T));
            PM_TRY(tmp.get(&run1, (size_t)T));
            PM_TRY(tmp.get(&hstart, (size_t)H + 1));
            PM_TRY(tmp.get(&cstart, (size_t)H + 1));
        }
        hipStream_t side[2];
        PM_HIP(side_streams(side));
        Fork fork(s, side, 2);
        PM_HIP(fork.status);
        if (cls[8] > cls[7]) {
            ProfScope pc("build_rows.b16384", side[1]);
            hipLaunchKernelGGL((k_rows_block<1024, 16>), dim3((unsigned)(cls[8] - cls[7])), dim3(1024), 0, side[1],
                               off_in, col_in, order, g->rank, g->off, n, cls[7], vbits, g->col, edge, ladder1, st);
        }
        if (cls[9] > cls[8]) {
            ProfScope pc("build_rows.b32768", side[1]);
            hipLaunchKernelGGL((k_rows_block_reg<1024, 32>), dim3((unsigned)(cls[9] - cls[8])), dim3(1024), 0,
                               side[1], off_in, col_in, order, g->rank, g->off, n, cls[8], vbits, g->col, edge,
                               ladder1, st);
        }
        if (T > 0) {
            // hub rows: chunks sorted in blocks, then merged within each row
            ProfScope pt("build_rows.hubs", side[0]);
            hipLaunchKernelGGL(k_hub_layout, dim3(1), dim3(kBlock), 0, side[0], g->off, rt, H, hstart, cstart);
            // each row has at most d / kHubChunk + 1 chunks
            const int64_t chunk_bound = T / kHubChunk + H;
            hipLaunchKernelGGL((k_hub_chunks<1024, 32>), dim3((unsigned)chunk_bound), dim3(1024), 0, side[0], off_in,
                               col_in, order, g->rank, hstart, cstart, n, rt, H, vbits, run0, st);
            // every hub row is longer than one chunk, so it takes at least one
            // round, and the round with L < degree <= 2L finishes it
            uint32_t *src = run0, *dst = run1;
            for (int64_t L = kHubChunk; L < (int64_t)g->dmax; L *= 2) {
                hipLaunchKernelGGL(k_hub_merge, dim3((unsigned)((T + kMergeTile - 1) / kMergeTile)), dim3(kBlock), 0,
                                   side[0], src, dst, T, hstart, H, L, rt, cls[kRowClasses], g->col, edge,
                                   ladder1);
                std::swap(src, dst);
            }
        }
        if (cls[1] > cls[0]) {
            ProfScope pc("build_rows.lane", s);
            hipLaunchKernelGGL(k_rows_group<16>, dim3((unsigned)((cls[1] - cls[0] + 15) / 16)), dim3(kBlock), 0, s,
                               off_in, col_in, order, g->rank, g->off, n, cls[0], cls[1], g->col, edge, ladder1,
                               st);
        }
        if (cls[2] > cls[1]) {
            ProfScope pc("build_rows.wave", s);
            hipLaunchKernelGGL(k_rows_group<64>, dim3((unsigned)((cls[2] - cls[1] + 3) / 4)), dim3(kBlock), 0, s,
                               off_in, col_in, order, g->rank, g->off, n, cls[1], cls[2], g->col, edge, ladder1,
                               st);
        }
        if (cls[3] > cls[2]) {
            ProfScope pc("build_rows.w128", s);
            hipLaunchKernelGGL(k_rows_bitonic<2>, dim3((unsigned)((cls[3] - cls[2] + 3) / 4)), dim3(kBlock), 0, s,
                               off_in, col_in, order, g->rank, g->off, n, cls[2], cls[3], g->col, edge, ladder1,
                               st);
        }
        if (cls[4] > cls[3]) {
            ProfScope pc("build_rows.w256", s);
            hipLaunchKernelGGL(k_rows_bitonic<4>, dim3((unsigned)((cls[4] - cls[3] + 3) / 4)), dim3(kBlock), 0, s,
                               off_in, col_in, order, g->rank, g->off, n, cls[3], cls[4], g->col, edge, ladder1,
                               st);
        }
        if (cls[5] > cls[4]) {
            ProfScope pc("build_rows.b1024", s);
            hipLaunchKernelGGL((k_rows_block_reg<64, 16>), dim3((unsigned)(cls[5] - cls[4])), dim3(64), 0, s, off_in,
                               col_in, order, g->rank, g->off, n, cls[4], vbits, g->col, edge, ladder1, st);
        }
        if (cls[6] > cls[5]) {
            ProfScope pc("build_rows.b4096", s);
            hipLaunchKernelGGL((k_rows_block_reg<256, 16>), dim3((unsigned)(cls[6] - cls[5])), dim3(256), 0, s, off_in,
                               col_in, order, g->rank, g->off, n, cls[5], vbits, g->col, edge, ladder1, st);
        }
        if (cls[7] > cls[6]) {
            ProfScope pc("build_rows.b8192", s);
            hipLaunchKernelGGL((k_rows_block_reg<512, 16>), dim3((unsigned)(cls[7] - cls[6])), dim3(512), 0, s, off_in,
                               col_in, order, g->rank, g->off, n, cls[6], vbits, g->col, edge, ladder1, st);
        }
        const hipError_t launched = hipGetLastError();
        PM_HIP(fork.join());  // before anything can return: the temporaries are released on s
        PM_HIP(launched);
    }
    tmp.release(vk0);
    tmp.release(vv0);
    tmp.release(vk1);
    tmp.release(vv1);
    // the reverse sort and the weights trust the columns: read the slot checks
    PM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (hst.err) {
        set_error(err_text(hst.err));
        return PM_EGRAPH;
    }
    for (int l = 2; l <= g->ladder_top; ++l) {
        const int64_t cnt = (int64_t)ladder_count(slots, l);
        hipLaunchKernelGGL(k_ladder_level, dim3(grid_for(cnt, kBlock, 1024)), dim3(kBlock), 0, s,
                           g->ladder + g->ladder_off[l - 1], cnt, g->ladder + g->ladder_off[l]);
        PM_HIP(hipGetLastError());
    }
    // the row hash of the adjacency tests (rows of degree <= 1024 many per
    // block, longer ones in windows; rows above 4096 have several windows)
    static_assert(kHashSmallBound == 1024, "row hash classes follow the row classes");
    PM_TRY(dev_alloc((void **)&g->hash, sizeof(uint32_t) * (2 * ss + kHashPad), s));
    g->bytes += sizeof(uint32_t) * (2 * ss + kHashPad);
    // built on a side stream (it reads only the finished rows) and joined back
    // before returning: the rows of degree <= 1024 beside the reverse sort,
    // the longer ones beside the weights pass, so that each of the two
    // shares the GPU with a part of the build
    hipStream_t hside[2];
    PM_HIP(side_streams(hside));
    Fork hfork(s, hside, 1);
    PM_HIP(hfork.status);
    // row classes 0, 5..8: degree above 0, 1024, 4096, 8192, 16384
    const int64_t hrows[5] = {cls[0], cls[5], cls[6], cls[7], cls[8]};
    const int64_t hslot_at[5] = {cls[kRowClasses + 1 + 0], cls[kRowClasses + 1 + 5], cls[kRowClasses + 1 + 6],
                                 cls[kRowClasses + 1 + 7], cls[kRowClasses + 1 + 8]};
    PM_TRY(build_rowhash(g, hrows, hslot_at, g->hash, hside[0], kRowHashSmall));

    uint32_t *ka, *kb, *vfree, *v2a;
    PM_TRY(tmp.get(&ka, ss));
    PM_TRY(tmp.get(&kb, ss));
    PM_TRY(tmp.get(&vfree, ss));
    PM_TRY(tmp.get(&v2a, ss));

    // reverse slots and the symmetry check: the slots' columns sorted stably,
    // with each slot's own position as payload (only the payload is kept)
    uint32_t *keys_unused, *rev;
    PM_TRY(radix_sort("reverse_sort", g->col, nullptr, kb, vfree, ka, v2a, slots, vbits, rscr, s, &keys_unused, &rev,
                      nullptr, nullptr, false));
    Fork hfork2(s, hside, 1);  // the side stream now also waits for the reverse sort
    PM_HIP(hfork2.status);
    PM_TRY(build_rowhash(g, hrows, hslot_at, g->hash, hside[0], kRowHashWide));

    // weights, their prefixes and the guide tables of the edge draws (nothing
    // below indexes memory through the weights until the checks are read back)
    const int64_t nseg = prefix_segments(slots);
    PM_TRY(dev_alloc((void **)&g->p_tau, sizeof(uint64_t) * ss, s));
    PM_TRY(dev_alloc((void **)&g->p_lam, sizeof(uint64_t) * ss, s));
    PM_TRY(dev_alloc((void **)&g->seg_tau, sizeof(uint64_t) * (nseg + 1), s));
    PM_TRY(dev_alloc((void **)&g->seg_lam, sizeof(uint64_t) * (nseg + 1), s));
    g->bytes += 2 * sizeof(uint64_t) * ss + 2 * sizeof(uint64_t) * (nseg + 1);
    const uint64_t gtarget = guide_target(slots);
    const uint64_t long_cap = gtarget / 64 + 2;
    PM_TRY(dev_alloc((void **)&g->guide_tau, sizeof(uint32_t) * (gtarget + 1), s));
    PM_TRY(dev_alloc((void **)&g->guide_lam, sizeof(uint32_t) * (gtarget + 1), s));
    g->bytes += 2 * sizeof(uint32_t) * (gtarget + 1);
    uint32_t *long_tau = nullptr, *long_lam = nullptr;
    PM_TRY(tmp.get(&long_tau, long_cap));
    PM_TRY(tmp.get(&long_lam, long_cap));
    if (slots == 0) {
        PM_TRY(fill_async<uint64_t>(g->seg_tau, 0ull, 1, s));
        PM_TRY(fill_async<uint64_t>(g->seg_lam, 0ull, 1, s));
    } else {
        U64x2 *sums = nullptr;
        char *scr = nullptr;
        PM_TRY(tmp.get(&sums, (size_t)nseg));
        PM_TRY(tmp.get(&scr, ScanScratch<U64x2>::bytes_for(nseg, 16)));
        ProfScope prof("weights_scan", s);
        const int64_t tiles = (slots + (int64_t)kBlock * kWItems - 1) / ((int64_t)kBlock * kWItems);
        {
            ProfScope pr("weights.reduce", s);
            hipLaunchKernelGGL(k_weights_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, s, edge, rev, g->off,
                               slots, g->p_tau, g->p_lam, g->rec, sums, st);
            PM_HIP(hipGetLastError());
        }
        PM_TRY((scan_launch<U64x2, 16>(SegIn{sums}, SegOut{g->seg_tau, g->seg_lam, nseg, &st->totals}, nseg,
                                       PairSumOp(), U64x2{0, 0}, scr, s)));
        hipLaunchKernelGGL(k_guide_setup, dim3(1), dim3(1), 0, s, st, slots, g->guide_tau, g->guide_lam);
        PM_HIP(hipGetLastError());
        {
            ProfScope pg("weights.guide", s);
            hipLaunchKernelGGL(k_guide_fill, dim3((unsigned)tiles), dim3(kBlock), 0, s, g->p_tau, g->p_lam,
                               g->seg_tau, g->seg_lam, slots, g->guide_tau, g->guide_lam, long_tau, long_lam,
                               (uint32_t)long_cap, st);
            PM_HIP(hipGetLastError());
        }
        const unsigned gl = (unsigned)std::min<uint64_t>(long_cap, 2048);
        hipLaunchKernelGGL(k_guide_long, dim3(gl), dim3(kBlock), 0, s, g->p_tau, g->seg_tau, &st->shift_tau,
                           g->guide_tau, long_tau, &st->nlong_tau, (uint32_t)long_cap, &st->err);
        hipLaunchKernelGGL(k_guide_long, dim3(gl), dim3(kBlock), 0, s, g->p_lam, g->seg_lam, &st->shift_lam,
                           g->guide_lam, long_lam, &st->nlong_lam, (uint32_t)long_cap, &st->err);
        PM_HIP(hipGetLastError());
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_n1, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, g->deg, n, st);
        PM_HIP(hipGetLastError());
    }
    PM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    // the scan writes its totals with the last segment offsets (seg[nseg]);
    // both stay 0 for an empty graph
    const uint64_t R[2] = {hst.totals.a, hst.totals.b};
    if (hst.err & ERR_ASYM) {
        set_error(err_text(hst.err));
        return PM_EGRAPH;
    }
    if (hst.err & (ERR_OVF_TAU | ERR_OVF_LAM)) {
        set_error(hst.err & ERR_OVF_TAU ? "2W does not fit in 64 bits" : "2 Lambda does not fit in 64 bits");
        return PM_EOVERFLOW;
    }
    if (hst.n1_hi != 0) {
        set_error("N1 does not fit in 64 bits");
        return PM_EOVERFLOW;
    }
    if (hst.err & ERR_GUIDE) {
        set_error("internal: guide table inconsistent with the weights");
        return PM_EDEVICE;
    }
    g->R_tau = R[0];
    g->R_lam = R[1];
    g->N1 = hst.n1_lo;
    g->isolated = (int64_t)hst.isolated;
    if (g->R_tau) {
        g->shift_tau = hst.shift_tau;
        g->nb_tau = ((g->R_tau - 1) >> g->shift_tau) + 1;
    }
    if (g->R_lam) {
        g->shift_lam = hst.shift_lam;
        g->nb_lam = ((g->R_lam - 1) >> g->shift_lam) + 1;
    }

    PM_HIP(hfork2.join());
    PM_HIP(hfork.join());
    PM_HIP(hipStreamSynchronize(s));
    guard.g = nullptr;
    *out = g;
    return PM_OK;
}

pm_status graph_export(const pm_graph *g, int64_t *off, int32_t *col, int32_t *rank, uint64_t *p_tau,
                       uint64_t *p_lam, hipStream_t s)
{
    if (!g) {
        set_error("null graph");
        return PM_EINVAL;
    }
    std::vector<uint32_t> off32;
    if (off) {
        off32.resize((size_t)g->n + 1);
        PM_HIP(hipMemcpyAsync(off32.data(), g->off, sizeof(uint32_t) * (g->n + 1), hipMemcpyDeviceToHost, s));
    }
    const int64_t nseg = prefix_segments(g->slots);
    std::vector<uint64_t> seg_t, seg_l;
    if (g->slots > 0) {
        if (col) PM_HIP(hipMemcpyAsync(col, g->col, sizeof(int32_t) * g->slots, hipMemcpyDeviceToHost, s));
        if (p_tau) {
            seg_t.resize((size_t)nseg);
            PM_HIP(hipMemcpyAsync(p_tau, g->p_tau, sizeof(uint64_t) * g->slots, hipMemcpyDeviceToHost, s));
            PM_HIP(hipMemcpyAsync(seg_t.data(), g->seg_tau, sizeof(uint64_t) * nseg, hipMemcpyDeviceToHost, s));
        }
        if (p_lam) {
            seg_l.resize((size_t)nseg);
            PM_HIP(hipMemcpyAsync(p_lam, g->p_lam, sizeof(uint64_t) * g->slots, hipMemcpyDeviceToHost, s));
            PM_HIP(hipMemcpyAsync(seg_l.data(), g->seg_lam, sizeof(uint64_t) * nseg, hipMemcpyDeviceToHost, s));
        }
    }
    if (rank && g->n > 0) PM_HIP(hipMemcpyAsync(rank, g->rank, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < off32.size(); ++i) off[i] = off32[i];  // the ABI's offsets are int64
    // the ABI's prefixes are global: segment prefix + the segment's offset
    for (size_t i = 0; i < (p_tau ? (size_t)g->slots : 0); ++i) p_tau[i] += seg_t[i >> kPrefixSegShift];
    for (size_t i = 0; i < (p_lam ? (size_t)g->slots : 0); ++i) p_lam[i] += seg_l[i >> kPrefixSegShift];
    return PM_OK;
}

}  // namespace pm

namespace pm {

pm_status graph_info(const pm_graph *g, pm_graph_info *out)
{
    if (!g || !out) {
        set_error("null argument");
        return PM_EINVAL;
    }
    out->n = g->n;
    out->m = g->slots / 2;
    out->dmax = g->dmax;
    out->isolated = g->isolated;
    out->W = g->R_tau / 2;
    out->Lambda = g->R_lam / 2;
    out->N1 = g->N1;
    out->device_bytes = g->bytes;
    return PM_OK;
}

}  // namespace pm
