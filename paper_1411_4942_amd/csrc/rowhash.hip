// Building the row hash (rowhash.hpp) of a prepared graph: every row's
// columns inserted into its own 2d entries by linear probing, in LDS.  Rows
// of degree at most kHashSmallBound are built many per block from a chunk of
// slots; longer rows in windows of kHashWin entries, one window per block
// (a row of at most kHashWin / 2 keys is one window).  A probe that runs past
// its window's end continues in the final table afterwards.
#include "graph.hpp"
#include "profile.hpp"
#include "rowhash.hpp"

namespace pm {

constexpr int kHashChunk = 2047;             // slots per block of the small-row kernel
constexpr int kHashSmall = kHashSmallBound;  // degree bound of the small-row kernel
// entries a small-row block can own: its rows start at most kHashChunk - 1
// slots into its chunk and end at most kHashSmall slots later (this bound and
// the chunk of 2047 slots keep the block's LDS within 32 KiB, so that five
// blocks share a CU)
constexpr int kHashSpan = 2 * (kHashChunk - 1 + kHashSmall);
// slots per thread of a small-row block: its rows start in one chunk, so they
// span fewer than kHashChunk + kHashSmall slots
constexpr int kHashRun = (kHashChunk + kHashSmall + kBlock - 1) / kBlock;
constexpr int kHashBatch = 8;  // keys a thread loads before handling them

// f(key) for the keys src[j], j in [j0, j1), this thread's share of the
// block (stride blockDim.x); kHashBatch keys are loaded before any of them
// is handled, so their loads overlap.  j1 < 2^31.
template <typename F>
__device__ __forceinline__ void for_keys(const uint32_t *__restrict__ src, uint32_t j0, uint32_t j1, F f)
{
    for (uint32_t base = j0 + threadIdx.x; base < j1; base += kHashBatch * blockDim.x) {
        uint32_t kv[kHashBatch];
#pragma unroll
        for (int q = 0; q < kHashBatch; ++q) {
            const uint32_t j = base + q * blockDim.x;
            kv[q] = j < j1 ? src[j] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kHashBatch; ++q)
            if (base + q * blockDim.x < j1) f(kv[q]);
    }
}

// insert key into the row's entries t[0, size) (LDS), probing from its home
__device__ __forceinline__ void lds_insert(uint32_t *t, uint32_t size, uint32_t key)
{
    uint32_t p = hash_home(key, size);
    for (uint32_t i = 0; i < size; ++i) {
        if (atomicCAS(&t[p], kHashEmpty, key) == kHashEmpty) return;
        p = p + 1 == size ? 0u : p + 1;
    }
}

// Rows with 1 <= d <= kHashSmall, whose first slot lies in this block's chunk
// [c kHashChunk, (c+1) kHashChunk) of the small rows' slots [0, s_end).
// Their entries form one span of at most kHashSpan, built in LDS.
__global__ __launch_bounds__(kBlock) void k_rowhash_small(const uint32_t *__restrict__ off,
                                                          const uint32_t *__restrict__ col, int64_t r_begin,
                                                          int64_t r_end, int64_t s_end, uint32_t *__restrict__ H)
{
    __shared__ uint32_t t[kHashSpan];  // its first two words carry the block's row range first
    __shared__ uint32_t roff[kHashChunk + 1];
    const int64_t s0 = (int64_t)blockIdx.x * kHashChunk;
    const int64_t s1 = s0 + kHashChunk < s_end ? s0 + kHashChunk : s_end;
    if (threadIdx.x < 2) {  // first row starting at or after s0 (resp. s1); rows < 2^31
        const int64_t target = threadIdx.x == 0 ? s0 : s1;
        int64_t lo = r_begin, hi = r_end;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)off[mid] >= target)
                hi = mid;
            else
                lo = mid + 1;
        }
        t[threadIdx.x] = (uint32_t)lo;
    }
    __syncthreads();
    // read before the barrier that precedes the table's first write
    const int64_t a0 = t[0], a1 = t[1];
    if (a0 >= a1) return;  // no row starts here (block-uniform)
    const int64_t nrows = a1 - a0;
    for (int64_t i = threadIdx.x; i <= nrows; i += blockDim.x) roff[i] = off[a0 + i];
    __syncthreads();
    const uint32_t first = roff[0];
    const uint32_t span = 2u * (roff[nrows] - first);
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) t[i] = kHashEmpty;
    __syncthreads();
    // each thread a run of consecutive slots: one search for the run's first
    // row, then the rows follow in order; the run's keys are loaded together
    // before the first insert
    const uint32_t nslots = roff[nrows] - first;
    const uint32_t per = (nslots + blockDim.x - 1) / blockDim.x;
    const uint32_t r0 = threadIdx.x * per, r1 = r0 + per < nslots ? r0 + per : nslots;
    if (r0 < r1) {
        uint32_t kv[kHashRun];
#pragma unroll
        for (int q = 0; q < kHashRun; ++q) kv[q] = r0 + q < r1 ? col[first + r0 + q] : 0u;
        int64_t lo = 0, hi = nrows;  // last row start <= first + r0
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (roff[mid] <= first + r0)
                lo = mid;
            else
                hi = mid;
        }
#pragma unroll
        for (int q = 0; q < kHashRun; ++q) {
            const uint32_t i = r0 + q;
            if (i >= r1) break;
            while (roff[lo + 1] <= first + i) ++lo;
            const uint32_t rb = roff[lo], d = roff[lo + 1] - rb;
            lds_insert(t + 2u * (rb - first), 2u * d, kv[q]);
        }
        for (uint32_t i = r0 + kHashRun; i < r1; ++i) {  // never taken while the bound above holds
            while (roff[lo + 1] <= first + i) ++lo;
            const uint32_t rb = roff[lo], d = roff[lo + 1] - rb;
            lds_insert(t + 2u * (rb - first), 2u * d, col[first + i]);
        }
    }
    __syncthreads();
    uint32_t *out = H + 2ull * first;
    for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) out[i] = t[i];
}

// Insert key into the row's global entries t[0, size), probing from p.
__device__ __forceinline__ void global_insert(uint32_t *t, uint32_t size, uint32_t p, uint32_t key)
{
    for (uint32_t i = 0; i < size; ++i) {
        if (atomicCAS(&t[p], kHashEmpty, key) == kHashEmpty) return;
        p = p + 1 == size ? 0u : p + 1;
    }
}

constexpr uint32_t kHashWin = 8192;     // entries per window (32 KB of LDS)
constexpr uint32_t kHashGroup = 8192;   // windows one counting pass over a row sorts out
constexpr uint32_t kSpillCap = 1u << 20;  // keys whose probe leaves their window

// Windows of the rows [r_begin, r_end) (degree above kHashSmallBound): row a
// has ceil(2 d / kHashWin) windows, numbered from wbase(a), an upper bound of
// the windows of the rows before it (gaps are allowed).
__device__ __forceinline__ uint64_t window_base(const uint32_t *off, int64_t r_begin, int64_t a)
{
    return 2ull * (off[a] - off[r_begin]) / kHashWin + (uint64_t)(a - r_begin);
}

__device__ __forceinline__ uint32_t window_count(uint32_t d)
{
    return (uint32_t)((2ull * d + kHashWin - 1) / kHashWin);
}

struct SpillList {
    uint32_t count;
    uint32_t overflow;
    uint32_t key[kSpillCap];
    uint32_t row[kSpillCap];   // row - r_begin
    uint32_t from[kSpillCap];  // entry (inside the row) where the probe goes on
};

// Rows with more than one window (r_sort on): the row's keys sorted out by
// window into its share of `part` (from the row's first slot less r_sort's;
// counting sort, kHashGroup windows per pass), and each window's first key
// position stored at wstart[wbase(a) + w].
__global__ __launch_bounds__(1024) void k_rowhash_sort(const uint32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ col, int64_t r_begin,
                                                       int64_t r_sort, uint32_t *__restrict__ part,
                                                       uint32_t *__restrict__ wstart)
{
    __shared__ uint32_t cnt[kHashGroup];
    const int64_t a = r_sort + blockIdx.x;
    const uint32_t rb = off[a], d = off[a + 1] - rb, size = 2u * d, nwin = window_count(d);
    const uint64_t wb = window_base(off, r_begin, a);
    uint32_t *keys = part + (rb - off[r_sort]);
    uint32_t placed = 0;  // keys of the groups before
    for (uint32_t g0 = 0; g0 < nwin; g0 += kHashGroup) {
        const uint32_t gw = nwin - g0 < kHashGroup ? nwin - g0 : kHashGroup;
        for (uint32_t i = threadIdx.x; i < gw; i += blockDim.x) cnt[i] = 0;
        __syncthreads();
        for_keys(col + rb, 0u, d, [&](uint32_t key) {
            const uint32_t w = hash_home(key, size) / kHashWin;
            if (w >= g0 && w - g0 < gw) atomicAdd(&cnt[w - g0], 1u);
        });
        __syncthreads();
        if (threadIdx.x == 0) {  // exclusive starts, kept as the scatter cursors
            uint32_t run = placed;
            for (uint32_t w = 0; w < gw; ++w) {
                const uint32_t c = cnt[w];
                cnt[w] = run;
                wstart[wb + g0 + w] = run;
                run += c;
            }
            placed = run;
        }
        __syncthreads();
        for_keys(col + rb, 0u, d, [&](uint32_t key) {
            const uint32_t w = hash_home(key, size) / kHashWin;
            if (w >= g0 && w - g0 < gw) keys[atomicAdd(&cnt[w - g0], 1u)] = key;
        });
        __syncthreads();  // (only thread 0's `placed` is used)
    }
}

// One window per block, over the window numbering of the rows [r_begin,
// r_end) (blocks in the gaps return at once).  A window's keys come from the
// row itself when the row has one window, else from the sorted-out `part`.
// A probe reaching the window's end goes to the spill list with the entry it
// continues from (the next window's first, or the row's first after the last).
__global__ __launch_bounds__(kBlock) void k_rowhash_window(const uint32_t *__restrict__ off,
                                                           const uint32_t *__restrict__ col, int64_t r_begin,
                                                           int64_t r_end, int64_t r_sort,
                                                           const uint32_t *__restrict__ part,
                                                           const uint32_t *__restrict__ wstart, SpillList *spill,
                                                           uint32_t *__restrict__ H)
{
    // 32 KiB in all, so that five blocks share a CU: the table's first word
    // carries the block's row first
    __shared__ uint32_t t[kHashWin];
    const uint64_t b = blockIdx.x;
    if (threadIdx.x == 0) {  // last row whose window base is <= b (rows < 2^31)
        int64_t lo = r_begin, hi = r_end;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (window_base(off, r_begin, mid) <= b)
                lo = mid;
            else
                hi = mid;
        }
        t[0] = (uint32_t)lo;
    }
    __syncthreads();
    const int64_t a = t[0];
    __syncthreads();  // every thread holds a before the table is cleared
    const uint32_t rb = off[a], d = off[a + 1] - rb, size = 2u * d, nwin = window_count(d);
    const uint64_t wb = window_base(off, r_begin, a);
    const uint32_t wi = (uint32_t)(b - wb);
    if (wi >= nwin) return;  // a gap (block-uniform)
    const uint32_t w0 = wi * kHashWin, wlen = size - w0 < kHashWin ? size - w0 : kHashWin;
    for (uint32_t i = threadIdx.x; i < wlen; i += blockDim.x) t[i] = kHashEmpty;
    __syncthreads();
    const uint32_t next = w0 + wlen == size ? 0u : w0 + wlen;
    const auto insert = [&](uint32_t key) {
        for (uint32_t p = hash_home(key, size) - w0; p < wlen; ++p)
            if (atomicCAS(&t[p], kHashEmpty, key) == kHashEmpty) return;
        const uint32_t c = atomicAdd(&spill->count, 1u);
        if (c < kSpillCap) {
            spill->key[c] = key;
            spill->row[c] = (uint32_t)(a - r_begin);
            spill->from[c] = next;
        } else {
            atomicOr(&spill->overflow, 1u);
        }
    };
    if (nwin == 1) {
        for_keys(col + rb, 0u, d, insert);
    } else {
        const uint32_t *keys = part + (rb - off[r_sort]);
        const uint32_t k0 = wstart[wb + wi], k1 = wi + 1 < nwin ? wstart[wb + wi + 1] : d;
        for_keys(keys, k0, k1, insert);
    }
    __syncthreads();
    uint32_t *out = H + 2ull * rb + w0;
    for (uint32_t i = threadIdx.x; i < wlen; i += blockDim.x) out[i] = t[i];
}

// The spilled keys go on probing in the finished table: every entry from
// their home to their window's end is taken, so this keeps the
// linear-probing invariant.
__global__ __launch_bounds__(kBlock) void k_rowhash_spill(const uint32_t *__restrict__ off, int64_t r_begin,
                                                          const SpillList *spill, uint32_t *__restrict__ H)
{
    const uint32_t n = spill->count < kSpillCap ? spill->count : kSpillCap;
    for (uint32_t i = (uint32_t)(blockIdx.x * blockDim.x + threadIdx.x); i < n; i += gridDim.x * blockDim.x) {
        const int64_t a = r_begin + spill->row[i];
        const uint32_t rb = off[a], size = 2u * (off[a + 1] - rb);
        global_insert(H + 2ull * rb, size, spill->from[i], spill->key[i]);
    }
}

// Only after a spill list overflow (not expected at load 1/2): every key of
// the rows [r_begin, r_end) missing from its row's table is inserted from its
// home.
__global__ __launch_bounds__(kBlock) void k_rowhash_repair(const uint32_t *__restrict__ off,
                                                           const uint32_t *__restrict__ col, int64_t r_begin,
                                                           const SpillList *spill, uint32_t *__restrict__ H)
{
    if (!spill->overflow) return;
    const int64_t a = r_begin + blockIdx.x;
    const uint32_t rb = off[a], d = off[a + 1] - rb, size = 2u * d;
    uint32_t *out = H + 2ull * rb;
    for (uint32_t j = threadIdx.x; j < d; j += blockDim.x) {
        const uint32_t key = col[rb + j];
        const uint32_t h = hash_home(key, size);
        bool present = false;
        for (uint32_t p = h, i = 0; i < size; ++i) {
            const uint32_t e = __hip_atomic_load(&out[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e == key) {
                present = true;
                break;
            }
            if (e == kHashEmpty) break;
            p = p + 1 == size ? 0u : p + 1;
        }
        if (!present) global_insert(out, size, h, key);
    }
}

// rows[c] = first row with degree above bound[c] of {0, kHashSmallBound,
// 4096, 8192, 16384}, slot_at[c] = that row's first slot (rows ascend by
// degree; rows before rows[0] have no slots).  H has 2 slots + kHashPad
// entries.  `parts` selects the rows built (kRowHashSmall, kRowHashWide);
// the two parts write disjoint entries and may run on different streams.
pm_status build_rowhash(const pm_graph *g, const int64_t rows[5], const int64_t slot_at[5], uint32_t *H,
                        hipStream_t s, int parts)
{
    const int64_t n = g->n, slots = g->slots;
    static_assert(2 * 4096 == kHashWin, "rows of degree up to 4096 are one window");
    ProfScope prof("rowhash", s);
    if (parts & kRowHashSmall) PM_TRY(fill_async<uint32_t>(H + 2 * slots, kHashEmpty, kHashPad, s));  // padding reads as empty
    const int64_t small_end = slot_at[1];
    if ((parts & kRowHashSmall) && small_end > 0) {
        ProfScope pc("rowhash.small", s);
        const int64_t blocks = (small_end + kHashChunk - 1) / kHashChunk;
        hipLaunchKernelGGL(k_rowhash_small, dim3((unsigned)blocks), dim3(kBlock), 0, s, g->off, g->col, rows[0],
                           rows[1], small_end, H);
        PM_HIP(hipGetLastError());
    }
    if ((parts & kRowHashWide) && n > rows[1]) {
        ProfScope pc("rowhash.wide", s);
        const int64_t r_begin = rows[1], r_sort = rows[2];  // rows above 1024; above 4096 (several windows)
        const int64_t wide_slots = slots - slot_at[1];
        const uint64_t nblocks = 2 * (uint64_t)wide_slots / kHashWin + (uint64_t)(n - r_begin) + 1;
        Temps tmp(s);
        uint32_t *part = nullptr, *wstart = nullptr;
        SpillList *spill = nullptr;
        PM_TRY(tmp.get(&part, (size_t)std::max<int64_t>(slots - slot_at[2], 1)));
        PM_TRY(tmp.get(&wstart, (size_t)nblocks));
        PM_TRY(tmp.get(&spill, 1));
        PM_TRY(fill_async<uint32_t>(&spill->count, 0u, 2, s));
        if (n > r_sort)
            hipLaunchKernelGGL(k_rowhash_sort, dim3((unsigned)(n - r_sort)), dim3(1024), 0, s, g->off, g->col, r_begin,
                               r_sort, part, wstart);
        hipLaunchKernelGGL(k_rowhash_window, dim3((unsigned)nblocks), dim3(kBlock), 0, s, g->off, g->col, r_begin, n,
                           r_sort, part, wstart, spill, H);
        hipLaunchKernelGGL(k_rowhash_spill, dim3(64), dim3(kBlock), 0, s, g->off, r_begin, spill, H);
        hipLaunchKernelGGL(k_rowhash_repair, dim3((unsigned)(n - r_begin)), dim3(kBlock), 0, s, g->off, g->col,
                           r_begin, spill, H);
        PM_HIP(hipGetLastError());
    }
    return PM_OK;
}

}  // namespace pm
