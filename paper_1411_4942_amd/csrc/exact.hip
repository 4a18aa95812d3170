// Exact induced 4-vertex counts on the device: ground truth at sizes the
// sampler runs at, split the way the paper describes its enumeration code
// (Section 6): the cycle-based subgraph counts by enumeration under the
// degree order, the others by formulas, then Eq. 1 solved for the induced
// counts.
//
// On the prepared graph vertex ids are ranks of the degree order and every
// row is ascending, so N+(x) (neighbours of higher rank) is the row suffix
// after position split[x] and the lower neighbours are the prefix.
//   N_1 = sum_v C(d_v, 3)                  (already in the prepared graph)
//   N_2 = W - 3T                           3-paths (W from the tau total)
//   N_3 = sum_v t_v (d_v - 2) = 1/2 sum_e t_e (d_u + d_v - 4)
//   N_4 = 4-cycles: at each cycle's highest vertex x, pairs of lower wedge
//         middles between x and each lower opposite vertex y
//   N_5 = sum_e C(t_e, 2)                  diamonds
//   N_6 = 4-cliques, counted at their lowest vertex u without listing them:
//         the graph induced on N+(u) as bit rows, a clique {u, v, w, x}
//         being a bit of row(v) & row(w) for an edge (v, w) inside N+(u)
// t_e = triangles on edge e (each found once, from its lowest vertex).
#include <algorithm>
#include <cstring>

#include "graph.hpp"
#include "profile.hpp"
#include "rowhash.hpp"

namespace pm {

pm_status check_device(const pm_graph *g);

namespace {

struct ExactAcc {
    unsigned long long tri;           // triangles (each once)
    unsigned long long k4;            // 4-cliques (each once)
    unsigned long long n3_lo, n3_hi;  // 2 N_3
    unsigned long long n5_lo, n5_hi;  // N_5
    unsigned long long n4_lo, n4_hi;  // N_4
};

// 128-bit accumulation from per-block partial sums
__device__ void add128(unsigned long long *lo, unsigned long long *hi, unsigned __int128 v)
{
    const unsigned long long l = (unsigned long long)v, h = (unsigned long long)(v >> 64);
    const unsigned long long old = atomicAdd(lo, l);
    const unsigned long long carry = (old + l < old) ? 1ull : 0ull;
    if (h + carry) atomicAdd(hi, h + carry);
}

// Sum of one 128-bit value per thread over the block, valid in thread 0.
// Every thread of the block must call it.
template <int THREADS>
__device__ unsigned __int128 block_sum128(unsigned __int128 v)
{
    __shared__ unsigned long long s_lo[THREADS], s_hi[THREADS];
    __syncthreads();  // a previous call's readers are done with the arrays
    s_lo[threadIdx.x] = (unsigned long long)v;
    s_hi[threadIdx.x] = (unsigned long long)(v >> 64);
    __syncthreads();
    for (int d = THREADS / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            const unsigned __int128 a = (unsigned __int128)s_lo[threadIdx.x] |
                                        ((unsigned __int128)s_hi[threadIdx.x] << 64);
            const unsigned __int128 b = (unsigned __int128)s_lo[threadIdx.x + d] |
                                        ((unsigned __int128)s_hi[threadIdx.x + d] << 64);
            const unsigned __int128 c = a + b;
            s_lo[threadIdx.x] = (unsigned long long)c;
            s_hi[threadIdx.x] = (unsigned long long)(c >> 64);
        }
        __syncthreads();
    }
    return (unsigned __int128)s_lo[0] | ((unsigned __int128)s_hi[0] << 64);
}

// Sum of one 64-bit value per lane over the wave, valid in lane 0.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
    return v;
}

// Sum of one 128-bit value per lane over the wave, valid in lane 0.
__device__ __forceinline__ unsigned __int128 wave_sum128(unsigned __int128 v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const unsigned long long lo = __shfl_down((unsigned long long)v, d, kWave);
        const unsigned long long hi = __shfl_down((unsigned long long)(v >> 64), d, kWave);
        v += (unsigned __int128)lo | ((unsigned __int128)hi << 64);
    }
    return v;
}

// split[x] = number of neighbours of x below x (rows ascending)
__global__ __launch_bounds__(kBlock) void k_split(const uint32_t *__restrict__ off, const uint32_t *__restrict__ col,
                                                  int64_t n, uint32_t *__restrict__ split)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = off[x], hi = off[x + 1];
        const int64_t a = lo;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (col[mid] < (uint32_t)x)
                lo = mid + 1;
            else
                hi = mid;
        }
        split[x] = (uint32_t)(lo - a);
    }
}

// Triangles and 4-cliques at their lowest vertex u, one u per block at a time
// (vertices with lo < d+(u) <= 32 W; W words of 32 bits per row).  Row i of
// the graph induced on N+(u) = {ids[0] < ids[1] < ...} has bit j when
// ids[i] ~ ids[j], j > i (only forward neighbours are looked up).
//  - Each bit is a triangle {u, v_i, v_j}, found once.  It adds one to t_e
//    of its three edges: (v_i, v_j) at the forward slot p of row v_i where
//    the lookup found v_j, and (u, v_i), (u, v_j) at u's own forward slots
//    (counted per member in the block, then added once per slot).
//  - A clique {u, v_i, v_j, v_k} (i < j < k) is bit k of row i & row j for
//    each bit j of row i, so each is counted once, by whole words.
// Rows and member counters live in LDS (`scratch` null) or, for long forward
// rows, in the block's slice of a global scratch array.  A member is found
// in an LDS hash of N+(u) (id -> index, at most half full: one or two
// reads) in the LDS classes, by binary search in the global one.
constexpr uint32_t kNoId = 0xFFFFFFFFu;  // an empty member-hash slot (vertex ids are below 2^31)

template <int W, bool GLOBAL, int THREADS>
__global__ __launch_bounds__(THREADS) void k_cliques(const uint32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ col,
                                                    const uint32_t *__restrict__ split, int64_t n, uint32_t lo_d,
                                                    uint32_t hi_d, uint32_t *__restrict__ scratch, uint32_t gslots,
                                                    uint32_t *__restrict__ t_e, ExactAcc *acc)
{
    constexpr int kLdsIds = GLOBAL ? 1 : 32 * W;
    constexpr int kLdsRows = GLOBAL ? 1 : 32 * W * W;
    constexpr uint32_t kSlots = GLOBAL ? 1 : 64 * W;  // member hash: twice the members
    __shared__ uint32_t s_ids[kLdsIds];
    __shared__ uint32_t s_tri[kLdsIds];  // triangles on (u, ids[i])
    __shared__ uint32_t s_rows[kLdsRows];
    __shared__ uint32_t h_key[kSlots];   // member id, or kNoId
    __shared__ uint16_t h_idx[kSlots];   // its index in ids
    // GLOBAL with gslots > 0: ids, their counters and a member hash of gslots
    // slots (a power of two >= 2 hi_d) in dynamic LDS; gslots = 0: ids and
    // counters in the block's global slice, members found by binary search
    extern __shared__ uint32_t dyn[];
    const uint32_t wd = GLOBAL ? (hi_d + 31) / 32 : (uint32_t)W;  // words per row
    const uint32_t slots = GLOBAL ? gslots : kSlots;
    uint32_t *const slice = GLOBAL ? scratch + (uint64_t)blockIdx.x * ((uint64_t)hi_d * wd + 2ull * hi_d) : nullptr;
    uint32_t *ids = GLOBAL ? (gslots ? dyn : slice) : s_ids;
    uint32_t *tri_u = GLOBAL ? ids + hi_d : s_tri;
    uint32_t *rows = GLOBAL ? slice + 2ull * hi_d : s_rows;
    uint32_t *hkey = GLOBAL ? dyn + 2ull * hi_d : h_key;
    uint16_t *hidx = GLOBAL ? reinterpret_cast<uint16_t *>(dyn + 2ull * hi_d + gslots) : h_idx;
    const int wv = threadIdx.x / kWave, lane = lane_id(), nwv = THREADS / kWave;
    unsigned long long k4 = 0, tri = 0;
    for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
        const uint32_t beg = off[u] + split[u], D = off[u + 1] - beg;
        if (D <= lo_d || D > hi_d) continue;  // block-uniform
        for (uint32_t i = threadIdx.x; i < D; i += THREADS) {
            ids[i] = col[beg + i];
            tri_u[i] = 0;
        }
        for (uint64_t i = threadIdx.x; i < (uint64_t)D * wd; i += THREADS) rows[i] = 0;
        if (GLOBAL) __threadfence();  // the cleared rows, before the atomics below
        if (slots) {
            for (uint32_t i = threadIdx.x; i < slots; i += THREADS) hkey[i] = kNoId;
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < D; i += THREADS) {  // D <= slots / 2: a free slot is always found
                const uint32_t key = ids[i];
                for (uint32_t h = hash_mix32(key) & (slots - 1);; h = (h + 1) & (slots - 1))
                    if (atomicCAS(&hkey[h], kNoId, key) == kNoId) {
                        hidx[h] = (uint16_t)i;
                        break;
                    }
            }
        }
        __syncthreads();
        // rows: each wave takes a member v_i and looks its forward neighbours up
        for (uint32_t i = wv; i < D; i += nwv) {
            const uint32_t v = ids[i];
            const uint32_t vb = off[v] + split[v], ve = off[v + 1];
            for (uint32_t p = vb + lane; p < ve; p += kWave) {
                const uint32_t x = col[p];
                uint32_t lo = D;  // x's index in ids (> i: x > v = ids[i]), D if absent
                if (!slots) {
                    uint32_t hi = D;
                    lo = i + 1;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (ids[mid] < x)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (lo < D && ids[lo] != x) lo = D;
                } else {
                    for (uint32_t h = hash_mix32(x) & (slots - 1);; h = (h + 1) & (slots - 1)) {
                        const uint32_t k = hkey[h];
                        if (k == x) {
                            lo = hidx[h];
                            break;
                        }
                        if (k == kNoId) break;
                    }
                }
                if (lo < D) {  // the triangle {u, v, x}
                    atomicOr(&rows[(uint64_t)i * wd + (lo >> 5)], 1u << (lo & 31));
                    ++tri;
                    atomicAdd(&t_e[p], 1u);  // (v, x)
                    atomicAdd(&tri_u[i], 1u);
                    atomicAdd(&tri_u[lo], 1u);
                }
            }
        }
        if (GLOBAL) __threadfence();  // the finished rows, before they are read back
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < D; i += THREADS)  // (u, ids[i]): other lowest vertices add here too
            if (tri_u[i]) atomicAdd(&t_e[beg + i], tri_u[i]);
        for (uint32_t i = threadIdx.x; i < D; i += THREADS) {
            const uint32_t *ri = rows + (uint64_t)i * wd;
            for (uint32_t wj = 0; wj < wd; ++wj) {
                uint32_t bits = ri[wj];
                while (bits) {
                    const uint32_t j = wj * 32 + (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1;
                    const uint32_t *rj = rows + (uint64_t)j * wd;
                    for (uint32_t w = j >> 5; w < wd; ++w) k4 += (unsigned long long)__popc(ri[w] & rj[w]);
                }
            }
        }
        __syncthreads();  // the rows are rebuilt for the next u
    }
    // per-wave sums (a block reduction's LDS would not fit beside the rows)
    k4 = wave_sum_u64(k4);
    tri = wave_sum_u64(tri);
    if (lane == 0 && k4) atomicAdd(&acc->k4, k4);
    if (lane == 0 && tri) atomicAdd(&acc->tri, tri);
}

// largest forward degree d+(u)
__global__ __launch_bounds__(kBlock) void k_dplus_max(const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ split, int64_t n,
                                                      uint32_t *__restrict__ out)
{
    uint32_t m = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t d = off[u + 1] - off[u] - split[u];
        m = d > m ? d : m;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(m, o, kWave);
        m = x > m ? x : m;
    }
    if (lane_id() == 0 && m) atomicMax(out, m);
}

// Sums over forward slots: 2 N_3 = sum t_e (d_u + d_v - 4), N_5 = sum C(t_e, 2)
__global__ __launch_bounds__(kBlock) void k_edge_sums(const uint32_t *__restrict__ off,
                                                      const SlotRec *__restrict__ rec,
                                                      const uint32_t *__restrict__ t_e, int64_t slots,
                                                      ExactAcc *acc)
{
    unsigned __int128 n3 = 0, n5 = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < slots;
         s += (int64_t)gridDim.x * blockDim.x) {
        const SlotRec e = rec[s];
        const uint32_t u = e.row, v = e.col;
        const uint64_t t = t_e[s];
        if (v <= u || t == 0) continue;
        const uint64_t du = (uint64_t)(off[u + 1] - off[u]), dv = e.cdeg;
        n3 += (unsigned __int128)t * (du + dv - 4);  // t > 0 means both degrees >= 2
        n5 += (unsigned __int128)(t * (t - 1) / 2);
    }
    n3 = block_sum128<kBlock>(n3);
    n5 = block_sum128<kBlock>(n5);
    if (threadIdx.x == 0) {
        if (n3) add128(&acc->n3_lo, &acc->n3_hi, n3);
        if (n5) add128(&acc->n5_lo, &acc->n5_hi, n5);
    }
}

// 4-cycles by the highest vertex x.  For each lower neighbour w of x and
// each lower neighbour y of w below x, the pair (x, y) gains a wedge; a pair
// with c wedges closes C(c, 2) 4-cycles at x.  Counted per x either in an LDS
// hash of the touched y (below) or in a counter array of n words per block.

constexpr int kC4Hash = 4096;  // LDS slots of the per-x wedge count table
constexpr uint32_t kC4Empty = 0xFFFFFFFFu;

// Vertices x in [0, x_end), one per block at a time, their wedge endpoints
// counted in an LDS open-addressing table.  An x with more than 3/4 of the
// table's slots in distinct endpoints is left to the global-array kernel
// (appended to `spill`).
__global__ __launch_bounds__(kBlock) void k_four_cycles_lds(const uint32_t *__restrict__ off,
                                                            const uint32_t *__restrict__ col,
                                                            const uint32_t *__restrict__ split, int64_t x_end,
                                                            uint32_t *__restrict__ spill, uint32_t *n_spill,
                                                            ExactAcc *acc)
{
    __shared__ uint32_t keys[kC4Hash];
    __shared__ uint32_t cnts[kC4Hash];
    __shared__ uint32_t touched[kC4Hash];
    __shared__ uint32_t s_nt, s_fail;
    const int w_id = threadIdx.x / kWave, lane = lane_id(), nw = kBlock / kWave;
    for (int i = threadIdx.x; i < kC4Hash; i += kBlock) {
        keys[i] = kC4Empty;
        cnts[i] = 0;
    }
    unsigned __int128 n4 = 0;
    for (int64_t x = blockIdx.x; x < x_end; x += gridDim.x) {
        const uint32_t lo_begin = off[x], lo_end = off[x] + split[x];
        if (lo_end - lo_begin < 2) continue;  // two wedges at least (block-uniform)
        if (threadIdx.x == 0) {
            s_nt = 0;
            s_fail = 0;
        }
        __syncthreads();
        for (uint32_t p = lo_begin + w_id; p < lo_end && !s_fail; p += nw) {
            const uint32_t w = col[p];  // w < x
            const uint32_t r0 = off[w], r1 = off[w + 1];
            for (uint32_t q = r0 + lane; q < r1; q += kWave) {
                const uint32_t y = col[q];
                if (y >= (uint32_t)x) break;  // rows ascending: the rest are higher too
                uint32_t h = hash_mix32(y) & (kC4Hash - 1);
                for (int t = 0; t < kC4Hash; ++t) {
                    const uint32_t k = keys[h];
                    if (k == y) {
                        atomicAdd(&cnts[h], 1u);
                        break;
                    }
                    if (k == kC4Empty) {
                        const uint32_t old = atomicCAS(&keys[h], kC4Empty, y);
                        if (old == kC4Empty) {
                            atomicAdd(&cnts[h], 1u);
                            const uint32_t nt = atomicAdd(&s_nt, 1u);
                            touched[nt] = h;
                            if (nt + 1 > kC4Hash * 3 / 4) s_fail = 1;
                            break;
                        }
                        if (old == y) {
                            atomicAdd(&cnts[h], 1u);
                            break;
                        }
                    }
                    h = (h + 1) & (kC4Hash - 1);
                }
            }
        }
        __syncthreads();
        const uint32_t nt = s_nt < (uint32_t)kC4Hash ? s_nt : (uint32_t)kC4Hash;
        const bool fail = s_fail != 0;
        for (uint32_t i = threadIdx.x; i < nt; i += kBlock) {
            const uint32_t h = touched[i];
            const uint64_t c = cnts[h];
            if (!fail) n4 += (unsigned __int128)(c * (c - 1) / 2);
            keys[h] = kC4Empty;
            cnts[h] = 0;
        }
        if (fail && threadIdx.x == 0) spill[atomicAdd(n_spill, 1u)] = (uint32_t)x;
        __syncthreads();  // the table is clear before the next x
    }
    n4 = block_sum128<kBlock>(n4);
    if (threadIdx.x == 0 && n4) add128(&acc->n4_lo, &acc->n4_hi, n4);
}

// Vertices x = n-1-b for b < n_top (the highest ids, hubs first), then the
// spilled ones; blocks take the next b from a queue, so the hubs' unequal
// work spreads over the blocks as it comes.  The opposite vertices y < x are
// counted one range of ids at a time in LDS: kC4Range 32-bit counters, or
// twice as many 16-bit ones when x has fewer than 2^16 lower neighbours (a
// pair's count never exceeds them).  Each lower neighbour w of x keeps a
// cursor into its row (rows ascend, so the entries of one range follow
// those of the range before): per range a lane reads the cursor and the id
// it points at, and walks the row's segment inside the range only when that
// id lies in it.  A row is thus read segment by
// segment, about once over all ranges, instead of one random counter update
// in global memory per wedge.  Lanes walk up to kC4LaneRun entries of a
// segment; longer segments go to an LDS queue that whole waves walk 64
// entries at a time.
constexpr int kC4Threads = 1024;
constexpr uint32_t kC4Range = 40448;  // LDS counters per range (all of a 160 KB LDS but the words below)
constexpr uint32_t kC4LongCap = 256;  // queued long segments per range
constexpr int kC4LaneRun = 16;        // entries a lane walks before queueing the rest of a segment
constexpr uint32_t kC4Inf = 0xFFFFFFFFu;

// state[i] of the i-th lower neighbour w of the current x: {cursor into row
// w, end of row w, id at the cursor (kC4Inf past the end), unused}
__global__ __launch_bounds__(kC4Threads) void k_four_cycles(const uint32_t *__restrict__ off,
                                                            const uint32_t *__restrict__ col,
                                                            const uint32_t *__restrict__ split, int64_t n,
                                                            int64_t n_top, const uint32_t *__restrict__ spill,
                                                            const uint32_t *n_spill, uint4 *__restrict__ state_all,
                                                            uint64_t cap, uint32_t *queue, ExactAcc *acc)
{
    __shared__ uint32_t cnt[kC4Range];
    __shared__ uint32_t longq[kC4LongCap];
    __shared__ uint32_t s_b, s_nlong;
    uint4 *state = state_all + (uint64_t)blockIdx.x * cap;
    const int tid = threadIdx.x, w_id = tid / kWave, lane = lane_id(), nw = kC4Threads / kWave;
    const int64_t total = n_top + (int64_t)*n_spill;
    for (uint32_t i = tid; i < kC4Range; i += kC4Threads) cnt[i] = 0;
    unsigned __int128 n4 = 0;
    for (;;) {
        if (tid == 0) s_b = atomicAdd(queue, 1u);
        __syncthreads();
        const int64_t b = s_b;
        __syncthreads();  // every thread has read s_b before thread 0 writes it again
        if (b >= total) break;  // block-uniform
        const uint32_t x = b < n_top ? (uint32_t)(n - 1 - b) : spill[b - n_top];
        const uint32_t lo = off[x], D = split[x];  // N-(x) = col[lo, lo + D)
        if (D < 2) continue;  // fewer than two wedges per pair (block-uniform)
        for (uint32_t i = tid; i < D; i += kC4Threads) {
            const uint32_t w = col[lo + i], c = off[w], e = off[w + 1];
            state[i] = make_uint4(c, e, c < e ? col[c] : kC4Inf, 0u);
        }
        // a pair's count is at most D: below 2^16, two 16-bit counters share a
        // word and a range spans twice the ids
        const bool half = D < 65536u;
        const uint32_t span = half ? 2 * kC4Range : kC4Range;
        const auto bump = [&](uint32_t y, uint32_t r0) {
            const uint32_t o = y - r0;
            if (half)
                atomicAdd(&cnt[o >> 1], 1u << ((o & 1u) << 4));
            else
                atomicAdd(&cnt[o], 1u);
        };
        for (uint32_t r0 = 0; r0 < x; r0 += span) {
            const uint32_t E = x - r0 < span ? x : r0 + span;  // this range: ids [r0, E)
            if (tid == 0) s_nlong = 0;
            __syncthreads();  // the state, the cleared counters and s_nlong are in place
            for (uint32_t i = tid; i < D; i += kC4Threads) {
                const uint4 st = state[i];
                if (st.z >= E) continue;  // nothing of row w in this range
                uint32_t p = st.x, nxt = kC4Inf;
                const uint32_t end = st.y;
                bool queued = false, lane_only = false;
                for (int taken = 0;;) {
                    uint32_t v[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = p + j < end ? col[p + j] : kC4Inf;
                    int j = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (j < q || v[q] >= E) continue;  // stop at the first id past the range
                        bump(v[q], r0);
                        j = q + 1;
                    }
                    p += j;
                    if (j < 4) {
                        nxt = v[j];  // the first id >= E, or kC4Inf past the row's end
                        break;
                    }
                    taken += 4;
                    if (!lane_only && taken >= kC4LaneRun) {
                        const uint32_t q = atomicAdd(&s_nlong, 1u);
                        if (q < kC4LongCap) {
                            longq[q] = i;
                            queued = true;
                            break;
                        }
                        lane_only = true;  // the queue is full: this lane walks on
                    }
                }
                state[i] = make_uint4(p, end, queued ? 0u : nxt, 0u);
            }
            __syncthreads();
            // the long segments, a wave each, 64 entries per step (a prefix of
            // each step's ids lies in the range: rows ascend)
            const uint32_t nl = s_nlong < kC4LongCap ? s_nlong : kC4LongCap;
            for (uint32_t q = w_id; q < nl; q += nw) {  // wave-uniform
                const uint32_t i = longq[q];
                const uint4 st = state[i];
                uint32_t p = st.x, nxt = kC4Inf;
                for (;;) {
                    const uint32_t idx = p + lane;
                    const uint32_t y = idx < st.y ? col[idx] : kC4Inf;
                    const bool in = y < E;
                    if (in) bump(y, r0);
                    const uint32_t c = (uint32_t)__popcll(__ballot(in));
                    p += c;
                    if (c < (uint32_t)kWave) {
                        nxt = __shfl(y, (int)c, kWave);
                        break;
                    }
                }
                if (lane == 0) state[i] = make_uint4(p, st.y, nxt, 0u);
            }
            __syncthreads();
            const uint32_t words = half ? (E - r0 + 1) / 2 : E - r0;
            for (uint32_t j = tid; j < words; j += kC4Threads) {
                const uint32_t wv = cnt[j];
                if (half) {
                    const uint64_t c0 = wv & 0xFFFFu, c1 = wv >> 16;
                    n4 += (unsigned __int128)(c0 * (c0 - 1) / 2 + c1 * (c1 - 1) / 2);
                } else {
                    const uint64_t c = wv;
                    n4 += (unsigned __int128)(c * (c - 1) / 2);
                }
                cnt[j] = 0;
            }
        }
    }
    n4 = wave_sum128(n4);
    if (lane == 0 && n4) add128(&acc->n4_lo, &acc->n4_hi, n4);
}

// first vertex with degree above `bound` (degrees ascend)
__global__ void k_first_above(const uint32_t *__restrict__ deg, int64_t n, uint32_t bound, int64_t *out)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (deg[mid] > bound)
            hi = mid;
        else
            lo = mid + 1;
    }
    *out = lo;
}

}  // namespace

pm_status exact_counts(const pm_graph *g, pm_exact *out, hipStream_t s)
{
    if (!g || !out) {
        set_error("exact_counts: null argument");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    std::memset(out, 0, sizeof(*out));
    const int64_t n = g->n, slots = g->slots;
    Temps tmp(s);
    ExactAcc *acc = nullptr;
    PM_TRY(tmp.get(&acc, 1));
    PM_TRY(fill_async<unsigned char>((unsigned char *)acc, 0, (int64_t)sizeof(ExactAcc), s));
    ProfScope prof_total("exact_total", s);
    if (slots > 0) {
        uint32_t *split = nullptr, *t_e = nullptr;
        PM_TRY(tmp.get(&split, (size_t)n));
        PM_TRY(tmp.get(&t_e, (size_t)slots));
        PM_TRY(fill_async<uint32_t>(t_e, 0u, slots, s));
        hipLaunchKernelGGL(k_split, dim3(grid_for(n, kBlock, 1 << 22)), dim3(kBlock), 0, s, g->off, g->col, n, split);
        {
            // triangles (with t_e) and 4-cliques by forward degree class:
            // rows in LDS up to 1024 members, in a global slice per block
            // above; vertices with fewer than two forward neighbours close
            // neither
            ProfScope prof("exact.triangles_cliques", s);
            uint32_t *dmax_d = nullptr;
            PM_TRY(tmp.get(&dmax_d, 1));
            PM_TRY(fill_async<uint32_t>(dmax_d, 0u, 1, s));
            hipLaunchKernelGGL(k_dplus_max, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, g->off, split, n,
                               dmax_d);
            uint32_t dmax = 0;
            PM_HIP(hipMemcpyAsync(&dmax, dmax_d, sizeof(dmax), hipMemcpyDeviceToHost, s));
            PM_HIP(hipStreamSynchronize(s));
            const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 8192));
            {
                ProfScope pc("exact.cliques.64", s);
                hipLaunchKernelGGL((k_cliques<2, false, kBlock>), dim3(grid), dim3(kBlock), 0, s, g->off, g->col, split, n,
                                   1u, 64u, nullptr, 0u, t_e, acc);
            }
            {
                ProfScope pc("exact.cliques.256", s);
                hipLaunchKernelGGL((k_cliques<8, false, kBlock>), dim3(grid), dim3(kBlock), 0, s, g->off, g->col, split, n,
                                   64u, 256u, nullptr, 0u, t_e, acc);
            }
            {
                ProfScope pc("exact.cliques.1024", s);
                hipLaunchKernelGGL((k_cliques<32, false, 1024>), dim3(grid), dim3(1024), 0, s, g->off, g->col, split, n,
                                   256u, 1024u, nullptr, 0u, t_e, acc);
            }
            if (dmax > 1024) {
                ProfScope pc("exact.cliques.global", s);
                const uint32_t wd = (dmax + 31) / 32;
                const uint64_t slice = ((uint64_t)dmax * wd + 2ull * dmax) * sizeof(uint32_t);
                // blocks with a slice each, at most 1 GiB of slices
                const unsigned gb = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(256, (1ull << 30) / slice));
                uint32_t *scr = nullptr;
                PM_TRY(tmp.get(&scr, (size_t)gb * ((size_t)dmax * wd + 2ull * dmax)));
                // ids, counters and the member hash in LDS when they fit in 64 KB
                uint32_t gslots = 1;
                while (gslots < 2 * dmax) gslots <<= 1;
                const size_t dyn = (2ull * dmax + gslots) * sizeof(uint32_t) + gslots * sizeof(uint16_t);
                const bool in_lds = dmax < 65536 && dyn <= (64u << 10);
                hipLaunchKernelGGL((k_cliques<1, true, 1024>), dim3(gb), dim3(1024), in_lds ? dyn : 0, s, g->off, g->col,
                                   split, n, 1024u, dmax, scr, in_lds ? gslots : 0u, t_e, acc);
            }
            hipLaunchKernelGGL(k_edge_sums, dim3(grid_for(slots, kBlock, 4096)), dim3(kBlock), 0, s, g->off, g->rec,
                               t_e, slots, acc);
            PM_HIP(hipGetLastError());
            tmp.release(t_e);
        }
        // 4-cycles: vertices of degree at most kC4LdsDegree in LDS tables,
        // the rest (and any whose table fills) range by range in LDS
        constexpr uint32_t kC4LdsDegree = 1024;
        ProfScope prof("exact.four_cycles", s);
        int64_t *xb_d = nullptr;
        uint32_t *spill = nullptr, *n_spill = nullptr;
        PM_TRY(tmp.get(&xb_d, 1));
        PM_TRY(tmp.get(&n_spill, 1));
        hipLaunchKernelGGL(k_first_above, dim3(1), dim3(1), 0, s, g->deg, n, kC4LdsDegree, xb_d);
        PM_TRY(fill_async<uint32_t>(n_spill, 0u, 1, s));
        int64_t x_big = 0;
        PM_HIP(hipMemcpyAsync(&x_big, xb_d, sizeof(x_big), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        PM_TRY(tmp.get(&spill, (size_t)std::max<int64_t>(x_big, 1)));
        if (x_big > 0)
            hipLaunchKernelGGL(k_four_cycles_lds, dim3((unsigned)std::min<int64_t>(x_big, 16384)), dim3(kBlock), 0, s,
                               g->off, g->col, split, x_big, spill, n_spill, acc);
        // one cursor state (16 bytes) per lower neighbour of the block's
        // current vertex: at most dmax, within a 4 GiB budget of blocks
        const uint64_t cap = (uint64_t)std::max<int64_t>(g->dmax, 1);
        const int blocks = (int)std::max<uint64_t>(
            1, std::min<uint64_t>(std::min<uint64_t>(256, (uint64_t)n), (4ull << 30) / (cap * sizeof(uint4))));
        uint4 *state = nullptr;
        uint32_t *queue = nullptr;
        PM_TRY(tmp.get(&state, (size_t)blocks * (size_t)cap));
        PM_TRY(tmp.get(&queue, 1));
        PM_TRY(fill_async<uint32_t>(queue, 0u, 1, s));
        hipLaunchKernelGGL(k_four_cycles, dim3(blocks), dim3(kC4Threads), 0, s, g->off, g->col, split, n, n - x_big,
                           spill, n_spill, state, cap, queue, acc);
        PM_HIP(hipGetLastError());
    }
    ExactAcc h;
    PM_HIP(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));

    typedef __int128 i128;
    typedef unsigned __int128 u128;
    const u128 n3x2 = (u128)h.n3_lo | ((u128)h.n3_hi << 64);
    const u128 n5 = (u128)h.n5_lo | ((u128)h.n5_hi << 64);
    const u128 n4 = (u128)h.n4_lo | ((u128)h.n4_hi << 64);
    const i128 N1 = (i128)g->N1, N2 = (i128)(g->R_tau / 2) - 3 * (i128)h.tri, N3 = (i128)(n3x2 / 2),
               N4 = (i128)n4, N5 = (i128)n5, N6 = (i128)h.k4;
    // Eq. 1 (N = A C) is upper triangular with unit diagonal; entry (i, j) is
    // the number of copies of motif i inside motif j
    const i128 c6 = N6;
    const i128 c5 = N5 - 6 * c6;
    const i128 c4 = N4 - c5 - 3 * c6;
    const i128 c3 = N3 - 4 * c5 - 12 * c6;
    const i128 c2 = N2 - 2 * c3 - 4 * c4 - 6 * c5 - 12 * c6;
    const i128 c1 = N1 - c3 - 2 * c5 - 4 * c6;
    const i128 Ns[7] = {0, N1, N2, N3, N4, N5, N6};
    const i128 Cs[7] = {0, c1, c2, c3, c4, c5, c6};
    for (int i = 1; i <= 6; ++i) {
        if (Cs[i] < 0 || Cs[i] >= ((i128)1 << 64) || Ns[i] < 0 || Ns[i] >= ((i128)1 << 64)) {
            set_error("exact_counts: a count does not fit in 64 bits");
            return PM_EOVERFLOW;
        }
        out->C[i] = (uint64_t)Cs[i];
        out->N[i] = (uint64_t)Ns[i];
    }
    out->triangles = h.tri;
    return PM_OK;
}

}  // namespace pm
