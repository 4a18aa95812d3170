// Graph preparation: validation, degrees, the degree-order relabel of
// Section 4, tau/lambda weights with their prefix sums (Sections 3 and 4),
// N_1 (Algorithm 2) and the guide tables of the edge draw.
//
// Relabel by two stable sorts and one transposition identity: with the rows
// placed in the new order (G1, columns mapped but unsorted), a stable sort of
// G1's entries by column yields them ordered by (column, row), which for a
// symmetric graph is exactly the new CSR with every row ascending (the
// transpose of a symmetric graph is itself).  A second stable sort of the
// result's slots by column lists, at position q, the slot holding the reverse
// of slot q: that permutation is at once the symmetry check and the reverse
// slot map the lambda weights need.
#include "graph.hpp"
#include "profile.hpp"
#include "radix.hpp"

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

__global__ void k_iota(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
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
    int64_t *off;  // writes off[i+1]
    __device__ __forceinline__ void operator()(int64_t i, uint64_t incl, uint64_t) const { off[i + 1] = (int64_t)incl; }
};

// Row holding slot p: upper_bound(off, p) - 1 over [lo, hi), all 64 lanes
// probing together (64-ary search); p is the same in every lane.
__device__ __forceinline__ int64_t wave_row_of(const int64_t *__restrict__ off, int64_t n, int64_t p)
{
    int64_t lo = 0, hi = n + 1;  // first x with off[x] > p lies in [lo, hi]
    const int lane = lane_id();
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t x = lo + (int64_t)(lane + 1) * step;
        const bool le = x < hi && off[x] <= p;
        const uint64_t m = __ballot(le);
        const int cnt = __popcll(m);  // probes at or below p form a prefix
        const int64_t nlo = lo + (int64_t)cnt * step;
        const int64_t nhi = lo + (int64_t)(cnt + 1) * step;
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;  // off[lo] <= p < off[lo + 1] (lo is the last x with off[x] <= p)
}

// G1: every input slot moved into the row of its vertex's new id, columns
// mapped to new ids (rows not yet sorted).  Slot-parallel: each wave owns
// 1024 consecutive slots (16 coalesced rows of 64); a 64-ary search brackets
// the rows they fall in, then each lane locates its slots' rows inside the
// bracket, its lower bound only moving forward.  The same pass checks every
// slot: column in range, no self-loop, strictly above the previous column of
// its row.  An out-of-range column is flagged and left unwritten (the caller
// stops on the flag).  Offsets were checked before this runs.
constexpr int kPlaceItems = 16;

__global__ __launch_bounds__(kBlock) void k_place_rows(const int64_t *__restrict__ off_in,
                                                       const int32_t *__restrict__ col_in, int64_t n, int64_t slots,
                                                       const int32_t *__restrict__ rank,
                                                       const int64_t *__restrict__ off_new,
                                                       uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                                                       PrepStats *st)
{
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int64_t span = (int64_t)kWave * kPlaceItems;
    const int64_t ranges = (slots + span - 1) / span;
    uint32_t err = 0;
    for (int64_t rg = wave; rg < ranges; rg += nwaves) {
        const int64_t p0 = rg * span;
        const int64_t plast = (p0 + span - 1 < slots) ? p0 + span - 1 : slots - 1;
        const int64_t ufirst = wave_row_of(off_in, n, p0);
        const int64_t ulast = wave_row_of(off_in, n, plast);
        int64_t lo0 = ufirst;  // rows of this lane's slots never decrease
#pragma unroll 4
        for (int i = 0; i < kPlaceItems; ++i) {
            const int64_t p = p0 + (int64_t)i * kWave + lane;
            if (p >= slots) break;
            // last u in [lo0, ulast] with off_in[u] <= p
            int64_t lo = lo0, hi = ulast + 1;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (off_in[mid] <= p)
                    lo = mid;
                else
                    hi = mid;
            }
            lo0 = lo;
            const int64_t u = lo, a = off_in[u];
            const int32_t c = col_in[p];
            if (c < 0 || (int64_t)c >= n) {
                err |= ERR_RANGE;
                continue;
            }
            if (c == (int32_t)u) err |= ERR_LOOP;
            if (p > a && col_in[p - 1] >= c) err |= ERR_ORDER;
            const int32_t ru = rank[u];
            const int64_t dst = off_new[ru] + (p - a);
            key[dst] = (uint32_t)rank[c];
            val[dst] = (uint32_t)ru;
        }
    }
    if (err) atomicOr(&st->err, err);
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
// both weights of every slot, parked in the prefix arrays, and one pair of
// sums per tile of kBlock * kWItems slots (the tiling of the apply launch).
// Each thread issues the loads of kWBatch items before any store, so their
// gathers overlap.
constexpr int kWItems = 16;
constexpr int kWBatch = 8;

__global__ __launch_bounds__(kBlock) void k_weights_reduce(const uint64_t *__restrict__ edge,
                                                           const uint32_t *__restrict__ rev,
                                                           const uint32_t *__restrict__ key2,
                                                           const int64_t *__restrict__ off, int64_t N,
                                                           uint64_t *__restrict__ p_tau,
                                                           uint64_t *__restrict__ p_lam, U64x2 *__restrict__ tile_sums,
                                                           PrepStats *st)
{
    __shared__ U64x2 s_wave[kBlock / kWave];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t wave_base = (int64_t)blockIdx.x * (kBlock * kWItems) + (int64_t)w * kWave * kWItems;
    uint32_t err = 0;
    uint64_t acc_t = 0, acc_l = 0;
#pragma unroll
    for (int h = 0; h < kWItems; h += kWBatch) {
        uint64_t e[kWBatch];
        uint32_t r[kWBatch], k2[kWBatch];
#pragma unroll
        for (int i = 0; i < kWBatch; ++i) {
            const int64_t idx = wave_base + (int64_t)(h + i) * kWave + lane;
            const bool ok = idx < N;
            e[i] = ok ? edge[idx] : 0ull;
            r[i] = ok ? rev[idx] : 0u;
            k2[i] = ok ? key2[idx] : 0u;
        }
        int64_t ou[kWBatch], ou1[kWBatch], ov[kWBatch], ov1[kWBatch];
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
            if (idx >= N) continue;
            const uint32_t u = (uint32_t)e[i];
            const int64_t rr = r[i];
            if (k2[i] != u) err |= ERR_ASYM;  // symmetry, half 1
            if (rr < ov[i] || rr >= ov1[i]) err |= ERR_ASYM;  // half 2
            const int64_t du = ou1[i] - ou[i], dv = ov1[i] - ov[i];
            const uint64_t tau = (uint64_t)(du - 1) * (uint64_t)(dv - 1);
            const uint64_t luv = (uint64_t)(du - 1 - (idx - ou[i]));
            const uint64_t lvu = (uint64_t)(dv - 1 - (rr - ov[i]));
            const uint64_t lam = luv * lvu;
            p_tau[idx] = tau;
            p_lam[idx] = lam;
            acc_t += tau;
            acc_l += lam;
        }
    }
    if (err) atomicOr(&st->err, err);
    const U64x2 acc = wave_reduce(U64x2{acc_t, acc_l}, PairSumOp());
    if (lane == 0) s_wave[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        U64x2 t{0, 0};
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) t = PairSumOp()(t, s_wave[i]);
        tile_sums[blockIdx.x] = t;
    }
}

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

// Launch 3 of the weights scan: the prefixes from the parked weights, the
// wrap checks and the guide entries.  Blocked arrangement: thread t of a tile
// owns kWItems consecutive slots, scans them sequentially, and only the
// thread totals go through a wave scan (one 64-lane scan per thread instead
// of one per item).  The tiles are those of k_weights_reduce.
__global__ __launch_bounds__(kBlock) void k_weights_apply(uint64_t *__restrict__ p_tau, uint64_t *__restrict__ p_lam,
                                                          int64_t N, const U64x2 *__restrict__ tile_prefix,
                                                          uint32_t *__restrict__ guide_tau,
                                                          uint32_t *__restrict__ guide_lam,
                                                          uint32_t *__restrict__ long_tau,
                                                          uint32_t *__restrict__ long_lam, uint32_t long_cap,
                                                          PrepStats *st)
{
    __shared__ U64x2 s_wave[kBlock / kWave];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t base = (int64_t)blockIdx.x * (kBlock * kWItems) + (int64_t)threadIdx.x * kWItems;
    const uint32_t sh_t = st->shift_tau, sh_l = st->shift_lam;
    const uint64_t nb_t = st->nb_tau, nb_l = st->nb_lam;
    uint64_t a[kWItems], b[kWItems];
    if (base + kWItems <= N) {
        // 128 contiguous bytes per array and thread, as 16-byte loads
        const uint4 *pa = reinterpret_cast<const uint4 *>(p_tau + base);
        const uint4 *pb = reinterpret_cast<const uint4 *>(p_lam + base);
#pragma unroll
        for (int i = 0; i < kWItems / 2; ++i) {
            const uint4 x = pa[i], y = pb[i];
            a[2 * i] = (uint64_t)x.x | ((uint64_t)x.y << 32);
            a[2 * i + 1] = (uint64_t)x.z | ((uint64_t)x.w << 32);
            b[2 * i] = (uint64_t)y.x | ((uint64_t)y.y << 32);
            b[2 * i + 1] = (uint64_t)y.z | ((uint64_t)y.w << 32);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kWItems; ++i) {
            a[i] = base + i < N ? p_tau[base + i] : 0ull;
            b[i] = base + i < N ? p_lam[base + i] : 0ull;
        }
    }
    // thread-local inclusive sums
#pragma unroll
    for (int i = 1; i < kWItems; ++i) {
        a[i] += a[i - 1];
        b[i] += b[i - 1];
    }
    // exclusive prefix of the thread inside the tile
    const U64x2 tot{a[kWItems - 1], b[kWItems - 1]};
    const U64x2 incl = wave_inclusive(tot, PairSumOp(), U64x2{0, 0});
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    U64x2 run = tile_prefix[blockIdx.x];
    for (int i = 0; i < w; ++i) run = PairSumOp()(run, s_wave[i]);
    run.a += incl.a - tot.a;
    run.b += incl.b - tot.b;
    uint32_t err = 0;
    uint64_t prev_a = run.a, prev_b = run.b;
#pragma unroll
    for (int i = 0; i < kWItems; ++i) {
        const int64_t idx = base + i;
        if (idx >= N) break;
        const uint64_t ia = run.a + a[i], ib = run.b + b[i];
        // the running sum passed 2^64 exactly where it decreases
        if (ia < prev_a) err |= ERR_OVF_TAU;
        if (ib < prev_b) err |= ERR_OVF_LAM;
        guide_fill(prev_a, ia, sh_t, nb_t, (uint32_t)idx, guide_tau, long_tau, long_cap, &st->nlong_tau, &st->err);
        guide_fill(prev_b, ib, sh_l, nb_l, (uint32_t)idx, guide_lam, long_lam, long_cap, &st->nlong_lam, &st->err);
        a[i] = ia;
        b[i] = ib;
        prev_a = ia;
        prev_b = ib;
    }
    if (base + kWItems <= N) {
        uint4 *pa = reinterpret_cast<uint4 *>(p_tau + base);
        uint4 *pb = reinterpret_cast<uint4 *>(p_lam + base);
#pragma unroll
        for (int i = 0; i < kWItems / 2; ++i) {
            pa[i] = make_uint4((uint32_t)a[2 * i], (uint32_t)(a[2 * i] >> 32), (uint32_t)a[2 * i + 1],
                               (uint32_t)(a[2 * i + 1] >> 32));
            pb[i] = make_uint4((uint32_t)b[2 * i], (uint32_t)(b[2 * i] >> 32), (uint32_t)b[2 * i + 1],
                               (uint32_t)(b[2 * i + 1] >> 32));
        }
    } else {
#pragma unroll
        for (int i = 0; i < kWItems; ++i)
            if (base + i < N) {
                p_tau[base + i] = a[i];
                p_lam[base + i] = b[i];
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

__global__ __launch_bounds__(kBlock) void k_guide_long(const uint64_t *__restrict__ P, const uint32_t *shift_p,
                                                       uint32_t *__restrict__ guide,
                                                       const uint32_t *__restrict__ long_list,
                                                       const uint32_t *nlong, uint32_t cap)
{
    const uint32_t shift = *shift_p;
    const uint64_t mask = (shift == 0) ? 0ull : ((1ull << shift) - 1ull);
    const uint32_t cnt = *nlong < cap ? *nlong : cap;  // listed runs were checked against nb
    for (uint32_t e = blockIdx.x; e < cnt; e += gridDim.x) {
        uint32_t s = long_list[e];
        uint64_t prev = s > 0 ? P[s - 1] : 0ull, cur = P[s];
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
    dev_free(g->off, s);
    dev_free(g->col, s);
    dev_free(g->edge, s);
    dev_free(g->ladder, s);
    dev_free(g->deg, s);
    dev_free(g->rank, s);
    dev_free(g->p_tau, s);
    dev_free(g->p_lam, s);
    dev_free(g->guide_tau, s);
    dev_free(g->guide_lam, s);
    delete g;
}

// Device bytes a prepared graph of n vertices and `slots` directed slots
// holds (what graph_create adds up in pm_graph::bytes).
uint64_t graph_bytes_for(int64_t n, int64_t slots)
{
    const uint64_t nn = (uint64_t)std::max<int64_t>(n, 1), ss = (uint64_t)std::max<int64_t>(slots, 1);
    uint64_t b = 4 * nn + 4 * nn + 8 * ((uint64_t)n + 1);
    const int top = ladder_top_for(slots);
    uint64_t total = 0;
    for (int l = 1; l <= top; ++l) total += (ladder_count(slots, l) + 31) / 32 * 32;
    if (top > 0) b += 4 * (total + 32);
    b += 12 * ss + 16 * ss;
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
    PM_TRY(dev_alloc((void **)&g->off, sizeof(int64_t) * (n + 1), s));
    g->bytes += sizeof(int32_t) * nn + sizeof(uint32_t) * nn + sizeof(int64_t) * (n + 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_rank_from_order, dim3(grid_stream(n)), dim3(kBlock), 0, s, order, g->rank, n);
        hipLaunchKernelGGL(k_copy_u32, dim3(grid_stream(n)), dim3(kBlock), 0, s, sorted_deg, g->deg, n);
        PM_HIP(hipGetLastError());
    }
    PM_TRY(fill_async<int64_t>(g->off, 0, 1, s));
    {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<uint64_t>::bytes_for(n, 16)));
        PM_TRY((scan_launch<uint64_t, 16>(DegIn{g->deg}, OffOut{g->off}, n, SumOp<uint64_t>(), 0ull, scr, s)));
    }
    tmp.release(vk0);
    tmp.release(vv0);
    tmp.release(vk1);
    tmp.release(vv1);

    const int vbits = bits_for(n > 0 ? (uint64_t)(n - 1) : 0);
    // the column buffers are padded to whole 128-byte lines (ladder level 0)
    const int64_t ssp = (ss + 31) / 32 * 32 + 32;
    uint32_t *ka, *va, *kb, *vb;
    PM_TRY(tmp.get(&ka, ss));
    PM_TRY(tmp.get(&va, ssp));
    PM_TRY(tmp.get(&kb, ss));
    PM_TRY(tmp.get(&vb, ssp));

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
    if (slots > 0) {
        ProfScope prof("place_rows", s);
        hipLaunchKernelGGL(k_place_rows, dim3(grid_for((slots + kPlaceItems - 1) / kPlaceItems, kBlock, 1 << 22)),
                           dim3(kBlock), 0, s, off_in, col_in, n, slots, g->rank, g->off, kb, vb, st);
        PM_HIP(hipGetLastError());
    }
    // the sorts and the weights trust the columns: read the slot checks
    PM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (hst.err) {
        set_error(err_text(hst.err));
        return PM_EGRAPH;
    }
    uint32_t *src_fin, *col_fin;
    PM_TRY(dev_alloc((void **)&g->edge, sizeof(uint64_t) * ss, s));
    // G1 sits in (kb, vb); the sort alternates (ka, va) and (kb, vb)
    PM_TRY(radix_sort("transpose_sort", kb, vb, ka, va, kb, vb, slots, vbits, rscr, s, &src_fin, &col_fin, g->edge,
                      g->ladder_top > 0 ? g->ladder + g->ladder_off[1] : nullptr));
    g->col = col_fin;
    tmp.keep(col_fin);
    for (int l = 2; l <= g->ladder_top; ++l) {
        const int64_t cnt = (int64_t)ladder_count(slots, l);
        hipLaunchKernelGGL(k_ladder_level, dim3(grid_for(cnt, kBlock, 1024)), dim3(kBlock), 0, s,
                           g->ladder + g->ladder_off[l - 1], cnt, g->ladder + g->ladder_off[l]);
        PM_HIP(hipGetLastError());
    }
    g->bytes += (sizeof(uint32_t) + sizeof(uint64_t)) * ss;
    uint32_t *vfree = (col_fin == va) ? vb : va;  // keys went into edge: ka, kb are free too
    uint32_t *v2a;
    PM_TRY(tmp.get(&v2a, ss));

    // reverse slots and the symmetry check: the slots' columns sorted stably,
    // with each slot's own position as payload
    uint32_t *key2, *rev;
    PM_TRY(radix_sort("reverse_sort", g->col, nullptr, kb, vfree, ka, v2a, slots, vbits, rscr, s, &key2, &rev));

    // weights, their prefixes and the guide tables of the edge draws (nothing
    // below indexes memory through the weights until the checks are read back)
    PM_TRY(dev_alloc((void **)&g->p_tau, sizeof(uint64_t) * ss, s));
    PM_TRY(dev_alloc((void **)&g->p_lam, sizeof(uint64_t) * ss, s));
    g->bytes += 2 * sizeof(uint64_t) * ss;
    const uint64_t gtarget = guide_target(slots);
    const uint64_t long_cap = gtarget / 64 + 2;
    PM_TRY(dev_alloc((void **)&g->guide_tau, sizeof(uint32_t) * (gtarget + 1), s));
    PM_TRY(dev_alloc((void **)&g->guide_lam, sizeof(uint32_t) * (gtarget + 1), s));
    g->bytes += 2 * sizeof(uint32_t) * (gtarget + 1);
    uint32_t *long_tau = nullptr, *long_lam = nullptr;
    PM_TRY(tmp.get(&long_tau, long_cap));
    PM_TRY(tmp.get(&long_lam, long_cap));
    {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<U64x2>::bytes_for(slots, 16)));
        ProfScope prof("weights_scan", s);
        auto mid = [&]() -> pm_status {
            hipLaunchKernelGGL(k_guide_setup, dim3(1), dim3(1), 0, s, st, slots, g->guide_tau, g->guide_lam);
            PM_HIP(hipGetLastError());
            return PM_OK;
        };
        if (slots > 0) {
            const int64_t tiles = (slots + (int64_t)kBlock * kWItems - 1) / ((int64_t)kBlock * kWItems);
            U64x2 *sums = (U64x2 *)scr;
            {
                ProfScope pr("weights.reduce", s);
                hipLaunchKernelGGL(k_weights_reduce, dim3((unsigned)tiles), dim3(kBlock), 0, s, g->edge, rev, key2,
                                   g->off, slots, g->p_tau, g->p_lam, sums, st);
            }
            hipLaunchKernelGGL((scan_tiles_kernel<U64x2, PairSumOp>), dim3(1), dim3(1024), 0, s, sums, tiles,
                               PairSumOp(), U64x2{0, 0}, &st->totals);
            PM_HIP(hipGetLastError());
            PM_TRY(mid());
            ProfScope pa("weights.apply", s);
            hipLaunchKernelGGL(k_weights_apply, dim3((unsigned)tiles), dim3(kBlock), 0, s, g->p_tau, g->p_lam, slots,
                               (const U64x2 *)sums, g->guide_tau, g->guide_lam, long_tau, long_lam,
                               (uint32_t)long_cap, st);
            PM_HIP(hipGetLastError());
        }
        if (slots > 0) {
            const unsigned gl = (unsigned)std::min<uint64_t>(long_cap, 2048);
            hipLaunchKernelGGL(k_guide_long, dim3(gl), dim3(kBlock), 0, s, g->p_tau, &st->shift_tau, g->guide_tau,
                               long_tau, &st->nlong_tau, (uint32_t)long_cap);
            hipLaunchKernelGGL(k_guide_long, dim3(gl), dim3(kBlock), 0, s, g->p_lam, &st->shift_lam, g->guide_lam,
                               long_lam, &st->nlong_lam, (uint32_t)long_cap);
            PM_HIP(hipGetLastError());
        }
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_n1, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, g->deg, n, st);
        PM_HIP(hipGetLastError());
    }
    uint64_t R[2] = {0, 0};
    if (slots > 0) {
        PM_HIP(hipMemcpyAsync(&R[0], g->p_tau + slots - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        PM_HIP(hipMemcpyAsync(&R[1], g->p_lam + slots - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    }
    PM_HIP(hipMemcpyAsync(&hst, st, sizeof(hst), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
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
    if (off) PM_HIP(hipMemcpyAsync(off, g->off, sizeof(int64_t) * (g->n + 1), hipMemcpyDeviceToHost, s));
    if (g->slots > 0) {
        if (col) PM_HIP(hipMemcpyAsync(col, g->col, sizeof(int32_t) * g->slots, hipMemcpyDeviceToHost, s));
        if (p_tau) PM_HIP(hipMemcpyAsync(p_tau, g->p_tau, sizeof(uint64_t) * g->slots, hipMemcpyDeviceToHost, s));
        if (p_lam) PM_HIP(hipMemcpyAsync(p_lam, g->p_lam, sizeof(uint64_t) * g->slots, hipMemcpyDeviceToHost, s));
    }
    if (rank && g->n > 0) PM_HIP(hipMemcpyAsync(rank, g->rank, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
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
