// Batched sampling: many prepared graphs, each with its own sample budgets,
// in one persistent launch over a table of work tiles, captured once as a
// HIP graph and replayed.
//
// A tile is (graph, sampler, first sample id, count, seed).  Every block
// takes tiles from a shared cursor until the table is exhausted, so graphs
// of very different sizes and budgets share the GPU without a launch each.
// Samples depend only on (seed, sampler, id): a graph's tallies equal those
// of its own pm_count with the same parameters, whatever the tiling.
//
// The replayed graph is: tile table and control block host -> device (from
// pinned buffers, so a new table needs no recapture), tallies zeroed by a
// kernel, the persistent kernel, tallies device -> host.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "batch.hpp"
#include "profile.hpp"
#include "sampler.hpp"

namespace pm {

pm_status finalize(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t W,
                   uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta, pm_result *out);
pm_status check_device(const pm_graph *g);
int sampler_cu_count(int dev);

__global__ __launch_bounds__(kBlock) void k_sample_batch(const BatchGraph *__restrict__ graphs,
                                                         const BatchTile *__restrict__ tiles, BatchCtl *ctl,
                                                         unsigned long long *__restrict__ tallies)
{
    __shared__ uint32_t s_tile;
    const uint32_t ntiles = ctl->ntiles, nlists = ctl->nlists;
    const uint32_t home = nlists ? blockIdx.x % nlists : 0u;
    uint32_t tried = 0;  // lists found exhausted (thread 0's)
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t t = ntiles;  // none left
            if (nlists == 0) {
                t = atomicAdd(&ctl->cursor, 1u);
            } else {
                while (tried < nlists) {
                    const uint32_t x = (home + tried) % nlists;
                    const uint32_t c = atomicAdd(&ctl->lcursor[x], 1u);
                    if (c < ctl->begin[x + 1] - ctl->begin[x]) {
                        t = ctl->begin[x] + c;
                        break;
                    }
                    ++tried;  // cursors only grow: this list stays exhausted
                }
            }
            s_tile = t;
        }
        __syncthreads();
        const uint32_t t = s_tile;
        __syncthreads();  // every thread has read s_tile before it is reused
        if (t >= ntiles) break;  // every block leaves once all its lists are exhausted
        const BatchTile T = tiles[t];
        uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
        for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
        if (T.tag == 0) {
            const SamplerView &g = graphs[T.graph].v[0];
            for (uint32_t i = threadIdx.x; i < T.count; i += blockDim.x)
                tally_add(cnt, sample_class<false>(g, T.seed, T.first + i));
        } else {
            const SamplerView &g = graphs[T.graph].v[1];
            for (uint32_t i = threadIdx.x; i < T.count; i += blockDim.x)
                tally_add(cnt, sample_class<true>(g, T.seed, T.first + i));
        }
        tally_flush(cnt, tallies + ((uint64_t)T.slot * 2 + T.tag) * PM_NUM_TALLIES);
    }
}

pm_status launch_tiles(const BatchGraph *graphs, const BatchTile *tiles, BatchCtl *ctl, uint64_t *tallies,
                       unsigned blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_sample_batch, dim3(blocks), dim3(kBlock), 0, s, graphs, tiles, ctl,
                       (unsigned long long *)tallies);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm

struct pm_batch {
    int device = 0;
    int32_t count = 0;
    std::vector<const pm_graph *> graphs;
    std::vector<pm_params> params;
    pm_tune tune{};
    uint32_t tile_cap = 0;
    uint32_t ntiles = 0;
    unsigned blocks = 0;
    pm::BatchGraph *d_graphs = nullptr;
    pm::BatchTile *d_tiles = nullptr, *h_tiles = nullptr;  // h_ pinned
    pm::BatchCtl *d_ctl = nullptr, *h_ctl = nullptr;
    uint64_t *d_tallies = nullptr, *h_tallies = nullptr;
    hipStream_t stream = nullptr;  // internal, default priority
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace pm {

namespace {

std::mutex g_tune_mu;
std::map<std::pair<int32_t, int>, pm_tune> g_tune_cache;  // (graphs, log2 samples) -> shape

uint64_t budget(const pm_graph *g, const pm_params &p, int tag)
{
    if (tag == 0) return g->R_tau ? p.k_path : 0;
    return g->R_lam ? p.k_cent : 0;
}

uint32_t tiles_needed(const std::vector<const pm_graph *> &gs, const std::vector<pm_params> &ps, uint32_t per)
{
    uint64_t n = 0;
    for (size_t i = 0; i < gs.size(); ++i)
        for (int tag = 0; tag < 2; ++tag) n += (budget(gs[i], ps[i], tag) + per - 1) / per;
    return n > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)n;
}

uint32_t fill_graph_tiles(pm_batch *b, int32_t i, uint32_t per, uint32_t n);

// The tile table: graphs dealt to kTileLists lists, largest budget first to
// the least loaded list; each list graph-major (consecutive tiles share a
// graph and its cached lines).
uint32_t fill_tiles(pm_batch *b, uint32_t per)
{
    std::vector<int32_t> order((size_t)b->count);
    for (int32_t i = 0; i < b->count; ++i) order[(size_t)i] = i;
    const auto work = [&](int32_t i) { return budget(b->graphs[i], b->params[i], 0) + budget(b->graphs[i], b->params[i], 1); };
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work(x) > work(y); });
    std::vector<std::vector<int32_t>> lists(kTileLists);
    uint64_t load[kTileLists] = {0};
    for (int32_t i : order) {
        uint32_t best = 0;
        for (uint32_t x = 1; x < kTileLists; ++x)
            if (load[x] < load[best]) best = x;
        lists[best].push_back(i);
        load[best] += work(i);
    }
    uint32_t n = 0;
    for (uint32_t x = 0; x < kTileLists; ++x) {
        b->h_ctl->begin[x] = n;
        b->h_ctl->lcursor[x] = 0;
        for (int32_t i : lists[x]) n = fill_graph_tiles(b, i, per, n);
    }
    b->h_ctl->begin[kTileLists] = n;
    b->h_ctl->nlists = kTileLists;
    return n;
}

uint32_t fill_graph_tiles(pm_batch *b, int32_t i, uint32_t per, uint32_t n)
{
    {
        for (int tag = 0; tag < 2; ++tag) {
            const uint64_t k = budget(b->graphs[i], b->params[i], tag);
            const uint64_t first = tag == 0 ? b->params[i].first_id_path : b->params[i].first_id_cent;
            for (uint64_t done = 0; done < k; done += per) {
                BatchTile &t = b->h_tiles[n++];
                t.graph = (uint32_t)i;
                t.tag = (uint32_t)tag;
                t.count = (uint32_t)std::min<uint64_t>(per, k - done);
                t.slot = (uint32_t)i;
                t.first = first + done;
                t.seed = b->params[i].seed;
            }
        }
    }
    return n;
}

pm_status check_params(const pm_params *p)
{
    if (p->k_path == 0 && p->k_cent == 0) {
        set_error("batch: a graph has k_path = k_cent = 0");
        return PM_EINVAL;
    }
    if (!(p->delta > 0.0 && p->delta < 1.0)) {
        set_error("batch: delta must lie in (0,1)");
        return PM_EINVAL;
    }
    return PM_OK;
}

void batch_free(pm_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    dev_free(b->d_graphs, b->stream);
    dev_free(b->d_tiles, b->stream);
    dev_free(b->d_ctl, b->stream);
    dev_free(b->d_tallies, b->stream);
    if (b->h_tiles) (void)hipHostFree(b->h_tiles);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    if (b->h_tallies) (void)hipHostFree(b->h_tallies);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
    delete b;
}

// the work of one run, enqueued on b->stream (captured or eager)
pm_status enqueue_run(pm_batch *b)
{
    PM_HIP(hipMemcpyAsync(b->d_tiles, b->h_tiles, sizeof(BatchTile) * b->tile_cap, hipMemcpyHostToDevice, b->stream));
    PM_HIP(hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, b->stream));
    PM_TRY(fill_async<uint64_t>(b->d_tallies, 0ull, (int64_t)b->count * 2 * PM_NUM_TALLIES, b->stream));
    PM_TRY(launch_tiles(b->d_graphs, b->d_tiles, b->d_ctl, b->d_tallies, b->blocks, b->stream));
    PM_HIP(hipMemcpyAsync(b->h_tallies, b->d_tallies, sizeof(uint64_t) * b->count * 2 * PM_NUM_TALLIES,
                          hipMemcpyDeviceToHost, b->stream));
    return PM_OK;
}

pm_status set_shape(pm_batch *b, const pm_tune &t)
{
    if (t.samples_per_tile < 64 || t.blocks_per_cu < 1 || t.blocks_per_cu > 64) {
        set_error("batch tune: samples_per_tile >= 64, blocks_per_cu in [1,64]");
        return PM_EINVAL;
    }
    const uint32_t need = tiles_needed(b->graphs, b->params, (uint32_t)t.samples_per_tile);
    if (need > b->tile_cap) {
        set_error("batch: tile table capacity exceeded");
        return PM_EINVAL;
    }
    b->tune = t;
    b->ntiles = fill_tiles(b, (uint32_t)t.samples_per_tile);
    b->h_ctl->ntiles = b->ntiles;
    b->h_ctl->cursor = 0;
    const uint64_t cap = (uint64_t)sampler_cu_count(b->device) * (uint64_t)t.blocks_per_cu;
    b->blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(cap, std::max<uint32_t>(b->ntiles, 1)));
    return PM_OK;
}

pm_status capture(pm_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    PM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    pm_status st = enqueue_run(b);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (st != PM_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (e != hipSuccess) {
        set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        return PM_EDEVICE;
    }
    b->graph = gr;
    PM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return PM_OK;
}

// time one eager run of the current shape (ms)
pm_status time_shape(pm_batch *b, float *ms)
{
    hipEvent_t a, z;
    PM_HIP(hipEventCreate(&a));
    PM_HIP(hipEventCreate(&z));
    PM_HIP(hipEventRecord(a, b->stream));
    pm_status st = enqueue_run(b);
    if (st == PM_OK) {
        PM_HIP(hipEventRecord(z, b->stream));
        PM_HIP(hipEventSynchronize(z));
        PM_HIP(hipEventElapsedTime(ms, a, z));
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    return st;
}

int log2_floor(uint64_t x)
{
    int l = 0;
    while (x > 1) {
        x >>= 1;
        ++l;
    }
    return l;
}

// Autotuner: the launch shape of this batch, measured.  Candidates are tile
// sizes {1024, 4096, 16384} x resident blocks per CU {2, 4, 8}; each is run
// once after a warm-up and the fastest kept.  Results are cached per (graph
// count, log2 of the total samples).
pm_status autotune(pm_batch *b, pm_tune *best)
{
    uint64_t total = 0;
    for (int32_t i = 0; i < b->count; ++i) total += budget(b->graphs[i], b->params[i], 0) + budget(b->graphs[i], b->params[i], 1);
    const std::pair<int32_t, int> key(b->count, log2_floor(total + 1));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *best = it->second;
            return PM_OK;
        }
    }
    const int tiles_c[3] = {1024, 4096, 16384};
    const int blocks_c[3] = {2, 4, 8};
    float best_ms = 1e30f;
    pm_tune bt{4096, 4};
    bool warm = false;
    for (int ti : tiles_c)
        for (int bl : blocks_c) {
            pm_tune t{ti, bl};
            if (tiles_needed(b->graphs, b->params, (uint32_t)ti) > b->tile_cap) continue;
            PM_TRY(set_shape(b, t));
            float ms = 0.f;
            if (!warm) {
                PM_TRY(time_shape(b, &ms));
                warm = true;
            }
            PM_TRY(time_shape(b, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                bt = t;
            }
        }
    *best = bt;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = bt;
    return PM_OK;
}

}  // namespace

pm_status batch_create(const pm_graph *const *graphs, const pm_params *params, int32_t count, const pm_tune *tune,
                       hipStream_t user_stream, pm_batch **out)
{
    if (!graphs || !params || !out || count <= 0) {
        set_error("batch: null argument or count <= 0");
        return PM_EINVAL;
    }
    *out = nullptr;
    for (int32_t i = 0; i < count; ++i) {
        if (!graphs[i]) {
            set_error("batch: null graph");
            return PM_EINVAL;
        }
        PM_TRY(check_device(graphs[i]));
        PM_TRY(check_params(&params[i]));
    }
    pm_batch *b = new (std::nothrow) pm_batch();
    if (!b) return PM_ENOMEM;
    struct Guard {
        pm_batch *b;
        ~Guard()
        {
            if (b) batch_free(b);
        }
    } guard{b};
    PM_HIP(hipGetDevice(&b->device));
    b->count = count;
    b->graphs.assign(graphs, graphs + count);
    b->params.assign(params, params + count);
    PM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    PM_HIP(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    PM_HIP(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    // order after the caller's stream (the graphs were prepared there)
    PM_HIP(hipEventRecord(b->ev_in, user_stream));
    PM_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));

    std::vector<BatchGraph> hg(count);
    for (int32_t i = 0; i < count; ++i) {
        hg[i].v[0] = view_of(graphs[i], false);
        hg[i].v[1] = view_of(graphs[i], true);
    }
    PM_TRY(dev_alloc((void **)&b->d_graphs, sizeof(BatchGraph) * count, b->stream));
    PM_HIP(hipMemcpyAsync(b->d_graphs, hg.data(), sizeof(BatchGraph) * count, hipMemcpyHostToDevice, b->stream));
    const uint32_t min_tile = (tune && tune->samples_per_tile > 0 && tune->samples_per_tile < 1024)
                                  ? (uint32_t)std::max<int32_t>(64, tune->samples_per_tile)
                                  : 1024u;
    b->tile_cap = std::max<uint32_t>(1, tiles_needed(b->graphs, b->params, min_tile));
    PM_TRY(dev_alloc((void **)&b->d_tiles, sizeof(BatchTile) * b->tile_cap, b->stream));
    PM_TRY(dev_alloc((void **)&b->d_ctl, sizeof(BatchCtl), b->stream));
    PM_TRY(dev_alloc((void **)&b->d_tallies, sizeof(uint64_t) * count * 2 * PM_NUM_TALLIES, b->stream));
    PM_HIP(hipHostMalloc((void **)&b->h_tiles, sizeof(BatchTile) * b->tile_cap, hipHostMallocDefault));
    PM_HIP(hipHostMalloc((void **)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault));
    PM_HIP(hipHostMalloc((void **)&b->h_tallies, sizeof(uint64_t) * count * 2 * PM_NUM_TALLIES,
                         hipHostMallocDefault));
    std::memset(b->h_tiles, 0, sizeof(BatchTile) * b->tile_cap);
    PM_HIP(hipStreamSynchronize(b->stream));  // descriptors uploaded before hg goes away

    pm_tune t{};
    if (tune && tune->samples_per_tile > 0) {
        t = *tune;
    } else {
        PM_TRY(autotune(b, &t));
    }
    PM_TRY(set_shape(b, t));
    PM_TRY(capture(b));
    guard.b = nullptr;
    *out = b;
    return PM_OK;
}

pm_status batch_set_params(pm_batch *b, const pm_params *params)
{
    if (!b || !params) {
        set_error("batch: null argument");
        return PM_EINVAL;
    }
    for (int32_t i = 0; i < b->count; ++i) PM_TRY(check_params(&params[i]));
    std::vector<pm_params> old = b->params;
    b->params.assign(params, params + b->count);
    PM_HIP(hipStreamSynchronize(b->stream));  // the previous replay has read the table
    pm_status st = set_shape(b, b->tune);
    if (st != PM_OK) {
        b->params = old;
        (void)set_shape(b, b->tune);
        return st;
    }
    return PM_OK;
}

pm_status batch_run(pm_batch *b, pm_result *out, hipStream_t user_stream)
{
    if (!b || !out) {
        set_error("batch: null argument");
        return PM_EINVAL;
    }
    PM_HIP(hipStreamSynchronize(b->stream));
    b->h_ctl->ntiles = b->ntiles;
    b->h_ctl->cursor = 0;
    PM_HIP(hipEventRecord(b->ev_in, user_stream));
    PM_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    {
        ProfScope prof("sample_batch", b->stream);
        PM_HIP(hipGraphLaunch(b->exec, b->stream));
    }
    PM_HIP(hipStreamSynchronize(b->stream));
    for (int32_t i = 0; i < b->count; ++i) {
        const pm_graph *g = b->graphs[i];
        const pm_params &p = b->params[i];
        const uint64_t *t = b->h_tallies + (size_t)i * 2 * PM_NUM_TALLIES;
        PM_TRY(finalize(t, t + PM_NUM_TALLIES, g->R_tau / 2, g->R_lam / 2, g->N1, p.k_path, p.k_cent, p.delta,
                        &out[i]));
    }
    return PM_OK;
}

pm_status batch_get_tune(const pm_batch *b, pm_tune *out)
{
    if (!b || !out) {
        set_error("batch: null argument");
        return PM_EINVAL;
    }
    *out = b->tune;
    return PM_OK;
}

pm_status batch_destroy(pm_batch *b)
{
    if (!b) {
        set_error("batch: null argument");
        return PM_EINVAL;
    }
    batch_free(b);
    return PM_OK;
}

}  // namespace pm
