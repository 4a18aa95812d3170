// The single-graph sampling kernels: Algorithm 1 (sample) classified as in
// Algorithm 2, and Algorithm 3 (sample-centered) classified as in Algorithm 4
// (the per-sample body is in sampler.hpp).  One lane per sample, grid-stride
// over sample ids; per-lane counters, one wave reduction and atomic per class.
#include "drawsort.hpp"
#include "graph.hpp"
#include "profile.hpp"
#include "sampler.hpp"
#include "streams.hpp"

#include <algorithm>
#include <atomic>
#include <mutex>

namespace pm {

static_assert(draw_sort_tiles(kSortedChunk) <= kDsMaxTiles, "a sort chunk fits the draw sort's column scan");

// U samples per lane per round of the grid-stride loop (U > 1 only
// unrolls the loop; each sample is independent).
template <bool CENTERED, int U, int SEARCH>
__global__ __launch_bounds__(kBlock) void k_sample(SamplerView g, uint64_t seed, uint64_t first, uint64_t k,
                                                   unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t base = 0; base < k; base += nthreads * U) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const uint64_t i = base + (uint64_t)q * nthreads + tid;
            if (i < k) tally_add(cnt, sample_class<CENTERED, SEARCH>(g, seed, first + i));
        }
    }
    tally_flush(cnt, tally);
}

// The same samples with the adjacency tests done by the wave together
// (ladder_contains_wave): the loop steps whole waves over the ids (over
// ids[j] when SORTED), so every lane stays in it until the wave's last
// round; lanes past k carry no sample.
template <bool CENTERED, bool SORTED>
__global__ __launch_bounds__(kBlock) void k_sample_wave(SamplerView g, uint64_t seed, uint64_t first, uint64_t k,
                                                        const uint32_t *__restrict__ ids,
                                                        unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
    const uint64_t lane = (uint64_t)lane_id();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
    for (uint64_t base = wave * kWave; base < k; base += nwaves * kWave) {  // wave-uniform
        const uint64_t j = base + lane;
        const bool act = j < k;
        const uint64_t id = first + (act ? (SORTED ? (uint64_t)ids[j] : j) : 0ull);
        const uint32_t cls = sample_class_wave<CENTERED>(g, seed, id, act);
        if (act) tally_add(cnt, cls);
    }
    tally_flush(cnt, tally);
}

// launch shape of the samplers (pm_set_sampler_shape)
static std::atomic<int> g_samples_per_lane{1};
static std::atomic<int> g_blocks_per_cu{4};
static std::atomic<int> g_draw_order{1};  // draw-ordered sampling for large k (pm_set_draw_order)
static std::atomic<uint64_t> g_draw_min{kSortedMinDefault};
static std::atomic<int> g_search_mode{PM_SEARCH_HASH};  // adjacency tests (pm_set_search_mode)

bool draw_order_enabled() { return g_draw_order.load() != 0; }
uint64_t draw_order_min() { return g_draw_min.load(); }

pm_status set_draw_order(int32_t enabled, uint64_t min_samples)
{
    g_draw_order.store(enabled ? 1 : 0);
    g_draw_min.store(min_samples ? min_samples : kSortedMinDefault);
    return PM_OK;
}

pm_status set_search_mode(int32_t mode)
{
    if (mode != PM_SEARCH_LANE && mode != PM_SEARCH_WAVE && mode != PM_SEARCH_HASH) {
        set_error("search mode: PM_SEARCH_LANE (0), PM_SEARCH_WAVE (1) or PM_SEARCH_HASH (2)");
        return PM_EINVAL;
    }
    g_search_mode.store(mode);
    return PM_OK;
}

pm_status set_sampler_shape(int32_t samples_per_lane, int32_t blocks_per_cu)
{
    if (!(samples_per_lane == 1 || samples_per_lane == 2 || samples_per_lane == 4) || blocks_per_cu < 1 ||
        blocks_per_cu > 64) {
        set_error("sampler shape: samples_per_lane in {1,2,4}, blocks_per_cu in [1,64]");
        return PM_EINVAL;
    }
    g_samples_per_lane.store(samples_per_lane);
    g_blocks_per_cu.store(blocks_per_cu);
    return PM_OK;
}

template <bool CENTERED, int U>
static void launch_k_sample(unsigned blocks, hipStream_t s, const SamplerView &v, uint64_t seed, uint64_t first,
                            uint64_t k, uint64_t *tally)
{
    if (g_search_mode.load() == PM_SEARCH_HASH)
        hipLaunchKernelGGL((k_sample<CENTERED, U, PM_SEARCH_HASH>), dim3(blocks), dim3(kBlock), 0, s, v, seed, first,
                           k, (unsigned long long *)tally);
    else
        hipLaunchKernelGGL((k_sample<CENTERED, U, PM_SEARCH_LANE>), dim3(blocks), dim3(kBlock), 0, s, v, seed, first,
                           k, (unsigned long long *)tally);
}

int sampler_cu_count(int dev)
{
    static std::mutex mu;
    static int cache[64] = {0};
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cache[dev] = c;
    }
    return cache[dev];
}

// Draw-ordered sampling.  Tallies are sums over sample ids, so the order in
// which samples run is free: sorting the ids of a chunk by the top
// kDrawKeyBits bits of their draw r lets neighbouring lanes read neighbouring
// guide entries, prefix lines, edge records and row-u data (r picks the
// slot), so a sample touches fewer distinct random lines.  Each sample then
// redraws its r from its id; tallies equal the unsorted kernel's exactly.

// the draw key of position i of a sort chunk: the top bits of the r of
// sample first + i
struct DrawKey {
    uint64_t R, seed, first;
    uint32_t tag;
    int kshift;
    __device__ uint32_t operator()(int64_t i) const
    {
        return (uint32_t)(draw_bounded(seed, tag, first + (uint64_t)i, R) >> kshift);
    }
};

template <bool CENTERED, int SEARCH>
__global__ __launch_bounds__(kBlock) void k_sample_sorted(SamplerView g, uint64_t seed, uint64_t first, uint64_t k,
                                                          const uint32_t *__restrict__ ids,
                                                          unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k; j += (uint64_t)gridDim.x * blockDim.x)
        tally_add(cnt, sample_class<CENTERED, SEARCH>(g, seed, first + ids[j]));
    tally_flush(cnt, tally);
}

// The ids [first, first + kc) sorted by their draw keys in b's buffers
// (kc <= b.chunk); *ids receives the sorted ids (minus first).
static pm_status sort_chunk(const SamplerView &v, bool centered, uint64_t seed, uint64_t first, uint64_t kc,
                            hipStream_t s, const DrawSortBufs &b, uint32_t **ids)
{
    const int rbits = bits_for(v.R - 1);  // r < R
    const int kshift = rbits > kDrawKeyBits ? rbits - kDrawKeyBits : 0;
    const int kbits = rbits - kshift;
    return draw_sort("draw_sort", DrawKey{v.R, seed, first, centered ? 1u : 0u, kshift}, kc, kbits, s, b, ids);
}

// The samples first + ids[j] for j < kc, into tally.
static pm_status sample_chunk(const SamplerView &v, bool centered, uint64_t seed, uint64_t first, uint64_t kc,
                              const uint32_t *ids, uint64_t *tally, unsigned blocks, hipStream_t s)
{
    const unsigned kb = (unsigned)std::min<uint64_t>((kc + kBlock - 1) / kBlock, blocks);
    unsigned long long *t = (unsigned long long *)tally;
    ProfScope pk(centered ? "sample_centered.sorted" : "sample_path.sorted", s);
    const int mode = g_search_mode.load();
    if (mode == PM_SEARCH_WAVE) {
        if (centered)
            hipLaunchKernelGGL((k_sample_wave<true, true>), dim3(kb), dim3(kBlock), 0, s, v, seed, first, kc, ids, t);
        else
            hipLaunchKernelGGL((k_sample_wave<false, true>), dim3(kb), dim3(kBlock), 0, s, v, seed, first, kc, ids, t);
    } else if (mode == PM_SEARCH_HASH) {
        if (centered)
            hipLaunchKernelGGL((k_sample_sorted<true, PM_SEARCH_HASH>), dim3(kb), dim3(kBlock), 0, s, v, seed, first,
                               kc, ids, t);
        else
            hipLaunchKernelGGL((k_sample_sorted<false, PM_SEARCH_HASH>), dim3(kb), dim3(kBlock), 0, s, v, seed, first,
                               kc, ids, t);
    } else if (centered)
        hipLaunchKernelGGL((k_sample_sorted<true, PM_SEARCH_LANE>), dim3(kb), dim3(kBlock), 0, s, v, seed, first, kc,
                           ids, t);
    else
        hipLaunchKernelGGL((k_sample_sorted<false, PM_SEARCH_LANE>), dim3(kb), dim3(kBlock), 0, s, v, seed, first, kc,
                           ids, t);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

static pm_status launch_sorted_in(const SamplerView &v, bool centered, uint64_t seed, uint64_t first, uint64_t k,
                                  uint64_t *tally, unsigned blocks, hipStream_t s, const DrawSortBufs &b)
{
    for (uint64_t c0 = 0; c0 < k; c0 += b.chunk) {
        const uint64_t kc = std::min(b.chunk, k - c0);
        uint32_t *ids = nullptr;
        PM_TRY(sort_chunk(v, centered, seed, first + c0, kc, s, b, &ids));
        PM_TRY(sample_chunk(v, centered, seed, first + c0, kc, ids, tally, blocks, s));
    }
    return PM_OK;
}

// buffers of one draw-order sort chunk of min(k, kSortedChunk) ids from tmp
static pm_status sort_bufs(Temps &tmp, uint64_t k, DrawSortBufs *b)
{
    const uint64_t chunk = std::min<uint64_t>(k, kSortedChunk);
    char *base = nullptr;
    PM_TRY(tmp.get(&base, draw_sort_bytes(chunk)));
    draw_sort_carve(base, chunk, b);
    return PM_OK;
}

// the draw-ordered launch with its buffers from the stream-ordered allocator
static pm_status launch_sorted(const SamplerView &v, bool centered, uint64_t seed, uint64_t first, uint64_t k,
                               uint64_t *tally, unsigned blocks, hipStream_t s)
{
    Temps tmp(s);
    DrawSortBufs b{};
    PM_TRY(sort_bufs(tmp, k, &b));
    return launch_sorted_in(v, centered, seed, first, k, tally, blocks, s, b);
}

// One sampler's k samples from id `first` into tally (device, added to).
// Draw-ordered launches take their buffers from `fixed` when given, else
// from the allocator.
static pm_status launch_sampler(const pm_graph *g, bool centered, uint64_t seed, uint64_t first, uint64_t k,
                                uint64_t *tally, hipStream_t s, const DrawSortBufs *fixed = nullptr)
{
    const SamplerView v = view_of(g, centered);
    if (v.R == 0 || k == 0) return PM_OK;
    const int U = g_samples_per_lane.load();
    const uint64_t want = (k + (uint64_t)kBlock * U - 1) / ((uint64_t)kBlock * U);
    const uint64_t cap = (uint64_t)sampler_cu_count(g->device) * (uint64_t)g_blocks_per_cu.load();
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
    ProfScope prof(centered ? "sample_centered" : "sample_path", s);
    if (k >= draw_order_min() && v.R > 1 && draw_order_enabled())
        return fixed ? launch_sorted_in(v, centered, seed, first, k, tally, (unsigned)cap, s, *fixed)
                     : launch_sorted(v, centered, seed, first, k, tally, (unsigned)cap, s);
    if (g_search_mode.load() == PM_SEARCH_WAVE) {
        const uint64_t wants = (k + kBlock - 1) / kBlock;
        const unsigned wb = (unsigned)std::max<uint64_t>(1, std::min(wants, cap));
        if (centered)
            hipLaunchKernelGGL((k_sample_wave<true, false>), dim3(wb), dim3(kBlock), 0, s, v, seed, first, k, nullptr,
                               (unsigned long long *)tally);
        else
            hipLaunchKernelGGL((k_sample_wave<false, false>), dim3(wb), dim3(kBlock), 0, s, v, seed, first, k,
                               nullptr, (unsigned long long *)tally);
        PM_HIP(hipGetLastError());
        return PM_OK;
    }
    switch (U * 2 + (centered ? 1 : 0)) {
    case 2: launch_k_sample<false, 1>(blocks, s, v, seed, first, k, tally); break;
    case 3: launch_k_sample<true, 1>(blocks, s, v, seed, first, k, tally); break;
    case 4: launch_k_sample<false, 2>(blocks, s, v, seed, first, k, tally); break;
    case 5: launch_k_sample<true, 2>(blocks, s, v, seed, first, k, tally); break;
    case 8: launch_k_sample<false, 4>(blocks, s, v, seed, first, k, tally); break;
    default: launch_k_sample<true, 4>(blocks, s, v, seed, first, k, tally); break;
    }
    PM_HIP(hipGetLastError());
    return PM_OK;
}

pm_status check_device(const pm_graph *g);

// The samplers' adjacency test over a list of pairs (each in the row of the
// smaller id, bounds from the offsets).
template <int SEARCH>
__global__ __launch_bounds__(kBlock) void k_adjacent(SamplerView g, const int32_t *__restrict__ a,
                                                     const int32_t *__restrict__ b, int64_t count,
                                                     uint8_t *__restrict__ out)
{
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    // wave-uniform loop (the cooperative search needs every lane)
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave;
    for (int64_t base = wave0; base < count; base += nthreads) {
        const int64_t i = base + lane_id();
        const bool act = i < count;
        SampleTests t;
        if (act) {
            const uint32_t x = (uint32_t)a[i], y = (uint32_t)b[i];
            const uint32_t lo = x < y ? x : y;
            t.lo[0] = g.off[lo];
            t.hi[0] = g.off[lo + 1];
            t.key[0] = x < y ? y : x;
        }
        uint32_t r;
        if (SEARCH == PM_SEARCH_WAVE)
            r = ladder_contains_wave(g.ladder, act, t.lo[0], t.hi[0], t.key[0]) ? 1u : 0u;
        else
            r = act ? row_contains<SEARCH>(g, t, 0) : 0u;
        if (act) out[i] = (uint8_t)r;
    }
}

pm_status adjacent(const pm_graph *g, const int32_t *a, const int32_t *b, int64_t count, uint8_t *out, int32_t mode,
                   hipStream_t s)
{
    if (!g || count < 0 || (count > 0 && (!a || !b || !out))) {
        set_error("adjacent: null argument or negative count");
        return PM_EINVAL;
    }
    if (mode != PM_SEARCH_LANE && mode != PM_SEARCH_WAVE && mode != PM_SEARCH_HASH) {
        set_error("adjacent: unknown search mode");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    if (count == 0) return PM_OK;
    const SamplerView v = view_of(g, false);
    const unsigned blocks = (unsigned)grid_for(count, kBlock, 1 << 16);
    if (mode == PM_SEARCH_HASH)
        hipLaunchKernelGGL((k_adjacent<PM_SEARCH_HASH>), dim3(blocks), dim3(kBlock), 0, s, v, a, b, count, out);
    else if (mode == PM_SEARCH_WAVE)
        hipLaunchKernelGGL((k_adjacent<PM_SEARCH_WAVE>), dim3(blocks), dim3(kBlock), 0, s, v, a, b, count, out);
    else
        hipLaunchKernelGGL((k_adjacent<PM_SEARCH_LANE>), dim3(blocks), dim3(kBlock), 0, s, v, a, b, count, out);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// The sorted ids of one draw-order sort chunk, copied to out (device).
pm_status draw_order(const pm_graph *g, int32_t centered, uint64_t seed, uint64_t first, uint64_t k, uint32_t *out,
                     hipStream_t s)
{
    if (!g || !out || k == 0 || k > kSortedChunk) {
        set_error("draw order: null argument, or k outside [1, 2^24]");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    const SamplerView v = view_of(g, centered != 0);
    if (v.R < 2) {
        set_error("draw order: the sampler's total weight is below 2");
        return PM_EINVAL;
    }
    Temps tmp(s);
    DrawSortBufs b{};
    PM_TRY(sort_bufs(tmp, k, &b));
    uint32_t *ids = nullptr;
    PM_TRY(sort_chunk(v, centered != 0, seed, first, k, s, b, &ids));
    PM_HIP(hipMemcpyAsync(out, ids, sizeof(uint32_t) * k, hipMemcpyDeviceToDevice, s));
    return PM_OK;
}

// Is a sampler's launch draw-ordered in a single sort chunk?
static bool one_sorted_chunk(const SamplerView &v, uint64_t k)
{
    return v.R > 1 && k > 0 && k >= draw_order_min() && draw_order_enabled() && k <= kSortedChunk;
}

// Both samplers draw-ordered in one chunk each: the centered sampler's keys
// are drawn and sorted on a side stream while the caller's stream sorts the
// 3-path sampler's; the side stream joins s before the 3-path samples, and
// the centered samples follow.  The two sorts are small launches that leave
// the GPU partly idle, so side by side they take less time than in turn
// (sorting the centered ids beside the 3-path sampling kernel instead slows
// that kernel by more than it saves).  Each sampler runs the same kernels on
// the same ids as in sequence, so the tallies are the same.
static pm_status sample_pair_overlapped(const pm_graph *g, const pm_params *p, uint64_t *tallies, hipStream_t s)
{
    const SamplerView vp = view_of(g, false), vc = view_of(g, true);
    const unsigned cap = (unsigned)((uint64_t)sampler_cu_count(g->device) * (uint64_t)g_blocks_per_cu.load());
    Temps tmp(s);
    DrawSortBufs bp{}, bc{};
    PM_TRY(sort_bufs(tmp, p->k_path, &bp));
    PM_TRY(sort_bufs(tmp, p->k_cent, &bc));
    hipStream_t side[2];
    PM_HIP(side_streams(side));
    uint32_t *ids_c = nullptr, *ids_p = nullptr;
    {
        ProfScope prof("draw_sorts", s);
        Fork fork(s, side, 1);  // joined before the temporaries are released on s
        PM_HIP(fork.status);
        PM_TRY(sort_chunk(vc, true, p->seed, p->first_id_cent, p->k_cent, side[0], bc, &ids_c));
        PM_TRY(sort_chunk(vp, false, p->seed, p->first_id_path, p->k_path, s, bp, &ids_p));
        // joined before the 3-path kernel: a sort still running beside it
        // slows it by more than the join costs
        PM_HIP(fork.join());
    }
    {
        ProfScope prof("sample_path", s);
        PM_TRY(sample_chunk(vp, false, p->seed, p->first_id_path, p->k_path, ids_p, tallies, cap, s));
    }
    ProfScope prof("sample_centered", s);
    return sample_chunk(vc, true, p->seed, p->first_id_cent, p->k_cent, ids_c, tallies + PM_NUM_TALLIES, cap, s);
}

pm_status sample_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, hipStream_t s)
{
    if (!g || !p || !tallies_dev) {
        set_error("null argument");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    PM_TRY(fill_async<uint64_t>(tallies_dev, 0ull, 2 * PM_NUM_TALLIES, s));
    if (one_sorted_chunk(view_of(g, false), p->k_path) && one_sorted_chunk(view_of(g, true), p->k_cent))
        return sample_pair_overlapped(g, p, tallies_dev, s);
    PM_TRY(launch_sampler(g, false, p->seed, p->first_id_path, p->k_path, tallies_dev, s));
    PM_TRY(launch_sampler(g, true, p->seed, p->first_id_cent, p->k_cent, tallies_dev + PM_NUM_TALLIES, s));
    return PM_OK;
}

__global__ void k_philox(const uint32_t *in, uint32_t *out, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint32_t *q = in + 6 * i;
    U32x4 r = philox4x32_10(U32x4{q[0], q[1], q[2], q[3]}, q[4], q[5]);
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

// Streaming copy, 16 bytes per lane per step: the reference kernel whose
// bytes are known exactly (calibrates hardware traffic counters, measures the
// streaming ceiling of the device).
__global__ __launch_bounds__(kBlock) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                       int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

pm_status device_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s)
{
    if ((bytes > 0 && (!dst || !src)) || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) {
        set_error("device_copy: device pointers aligned to 16 bytes, size a multiple of 16");
        return PM_EINVAL;
    }
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return PM_OK;
    ProfScope prof("stream_copy", s);
    hipLaunchKernelGGL(k_stream_copy, dim3(grid_for(n, kBlock, 1 << 22)), dim3(kBlock), 0, s, (const uint4 *)src,
                       (uint4 *)dst, n);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

// Independent random 4-byte loads from a table: the ceiling for line-granular
// random access (each load touches its own line).  Indices come from a
// splitmix64 stream; the XOR of the loaded words keeps the loads live.
__global__ __launch_bounds__(kBlock) void k_random_gather(const uint32_t *__restrict__ table, uint64_t words,
                                                         int64_t count, uint64_t seed,
                                                         unsigned long long *__restrict__ sink)
{
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        acc ^= table[z % words];
    }
    const uint32_t r = wave_sum_u32(acc);  // keeps every load; the value itself is not used
    if (lane_id() == 0 && r == 0xFFFFFFFFu) atomicAdd(sink, 1ull);
}

pm_status device_gather(const void *table, uint64_t bytes, int64_t count, uint64_t seed, hipStream_t s)
{
    if (!table || bytes < 4 || count < 0 || ((uintptr_t)table & 3u) != 0) {
        set_error("device_gather: device table of at least 4 bytes, 4-byte aligned, count >= 0");
        return PM_EINVAL;
    }
    if (count == 0) return PM_OK;
    unsigned long long *sink = nullptr;
    PM_TRY(dev_alloc((void **)&sink, sizeof(unsigned long long), s));
    {
        ProfScope prof("random_gather", s);
        hipLaunchKernelGGL(k_random_gather, dim3(grid_for(count, kBlock, 1 << 22)), dim3(kBlock), 0, s,
                           (const uint32_t *)table, bytes / 4, count, seed, sink);
    }
    hipError_t e = hipGetLastError();
    dev_free(sink, s);
    if (e != hipSuccess) {
        set_error(std::string("device_gather: ") + hipGetErrorString(e));
        return PM_EDEVICE;
    }
    return PM_OK;
}

pm_status philox_device(const uint32_t *in, uint32_t *out, int64_t count)
{
    if (count < 0 || (count > 0 && (!in || !out))) {
        set_error("bad arguments");
        return PM_EINVAL;
    }
    if (count == 0) return PM_OK;
    hipStream_t s = nullptr;
    uint32_t *din = nullptr, *dout = nullptr;
    PM_TRY(dev_alloc((void **)&din, sizeof(uint32_t) * 6 * count, s));
    pm_status st = dev_alloc((void **)&dout, sizeof(uint32_t) * 4 * count, s);
    if (st != PM_OK) {
        dev_free(din, s);
        return st;
    }
    hipError_t e = hipMemcpyAsync(din, in, sizeof(uint32_t) * 6 * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, din, dout, count);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(uint32_t) * 4 * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(din, s);
    dev_free(dout, s);
    if (e != hipSuccess) {
        set_error(std::string("philox_device: ") + hipGetErrorString(e));
        return PM_EDEVICE;
    }
    return PM_OK;
}

}  // namespace pm

namespace pm {

pm_status finalize(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t W,
                   uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta, pm_result *out);

pm_status check_device(const pm_graph *g)
{
    int dev = -1;
    PM_HIP(hipGetDevice(&dev));
    if (dev != g->device) {
        set_error("graph lives on device " + std::to_string(g->device) + ", current device is " +
                  std::to_string(dev));
        return PM_EINVAL;
    }
    return PM_OK;
}

// Run both samplers of one graph through `run` (which fills 2 x PM_NUM_TALLIES
// device tallies), read the tallies back and finalize.
pm_status count_with(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s,
                     pm_status (*run)(const pm_graph *, const pm_params *, uint64_t *, hipStream_t))
{
    if (!g || !p || !out) {
        set_error("null argument");
        return PM_EINVAL;
    }
    if (p->k_path == 0 && p->k_cent == 0) {
        set_error("k_path and k_cent are both 0");
        return PM_EINVAL;
    }
    if (!(p->delta > 0.0 && p->delta < 1.0)) {
        set_error("delta must lie in (0,1)");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    uint64_t *t = nullptr;
    PM_TRY(dev_alloc((void **)&t, 2 * PM_NUM_TALLIES * sizeof(uint64_t), s));
    uint64_t host[2 * PM_NUM_TALLIES];
    pm_status st = run(g, p, t, s);
    if (st == PM_OK) {
        hipError_t e = hipMemcpyAsync(host, t, sizeof(host), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error(std::string("pm_count: ") + hipGetErrorString(e));
            st = PM_EDEVICE;
        }
    }
    dev_free(t, s);
    if (st != PM_OK) return st;
    return finalize(host, host + PM_NUM_TALLIES, g->R_tau / 2, g->R_lam / 2, g->N1, p->k_path, p->k_cent, p->delta,
                    out);
}

pm_status count_on_graph(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s)
{
    return count_with(g, p, out, s, sample_async);
}

// ---------------------------------------------------------------------------
// pm_count_noalloc: pm_count with its device scratch in a fixed array of the
// library (for callers that cannot allocate).  The array holds both
// samplers' tallies and the buffers of one draw-order sort chunk of
// kStaticChunk ids; larger budgets are sorted and sampled chunk by chunk.
// Each device the library runs on keeps its own copy of the array for the
// life of the process; every call on a device shares it.
// ---------------------------------------------------------------------------

constexpr uint64_t kStaticChunk = 1ull << 22;
constexpr size_t kStaticTallyBytes = 256;  // 2 x PM_NUM_TALLIES u64, padded to 256
constexpr size_t kStaticScratchBytes = kStaticTallyBytes + draw_sort_bytes(kStaticChunk);
static_assert(2 * PM_NUM_TALLIES * sizeof(uint64_t) <= kStaticTallyBytes, "tallies fit their slice");

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// the device address of this device's copy of `scratch` (looked up once per
// device, with that device current; host code never uses the symbol's name
// as an address)
static pm_status scratch_on_device(int dev, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *ptr[64] = {nullptr};
    if (dev < 0 || dev >= 64) {
        set_error("pm_count_noalloc: device index out of range");
        return PM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("pm_count_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return PM_EDEVICE;
        }
        ptr[dev] = (unsigned char *)p;
    }
    *out = ptr[dev];
    return PM_OK;
}

size_t static_scratch_bytes() { return kStaticScratchBytes; }

pm_status count_noalloc(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s)
{
    if (!g || !p || !out) {
        set_error("null argument");
        return PM_EINVAL;
    }
    if (p->k_path == 0 && p->k_cent == 0) {
        set_error("k_path and k_cent are both 0");
        return PM_EINVAL;
    }
    if (!(p->delta > 0.0 && p->delta < 1.0)) {
        set_error("delta must lie in (0,1)");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    unsigned char *base = nullptr;
    PM_TRY(scratch_on_device(g->device, &base));
    uint64_t *tally = reinterpret_cast<uint64_t *>(base);
    DrawSortBufs b{};
    draw_sort_carve(base + kStaticTallyBytes, kStaticChunk, &b);
    // the tallies keep the last call's contents: clear them (a fill kernel)
    PM_TRY(fill_async<uint64_t>(tally, 0ull, 2 * PM_NUM_TALLIES, s));
    PM_TRY(launch_sampler(g, false, p->seed, p->first_id_path, p->k_path, tally, s, &b));
    PM_TRY(launch_sampler(g, true, p->seed, p->first_id_cent, p->k_cent, tally + PM_NUM_TALLIES, s, &b));
    uint64_t host[2 * PM_NUM_TALLIES];
    hipError_t e = hipMemcpyAsync(host, tally, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("pm_count_noalloc: ") + hipGetErrorString(e));
        return PM_EDEVICE;
    }
    return finalize(host, host + PM_NUM_TALLIES, g->R_tau / 2, g->R_lam / 2, g->N1, p->k_path, p->k_cent, p->delta,
                    out);
}

}  // namespace pm
