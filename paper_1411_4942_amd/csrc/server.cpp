// Served mode: a request loop with continuous batching.
//
// One worker thread per server runs steps.  A step is one launch of the
// persistent tile kernel over a chunk of every active request's remaining
// ids; while it runs on the step stream the worker admits queued requests
// (first come, first served) and prepares the graphs they need on a second
// stream, so preparation overlaps sampling and new requests join the next
// step.  Admission needs a free slot and the graph resident: a graph that is
// not is prepared if its footprint fits the HBM budget, after evicting idle
// resident graphs least recently used first.  A request that asks for a
// relative error runs a pilot of k_pilot ids per sampler first; its budgets
// are then sized with Corollary 5.3 (samples_for_request) and the remaining
// ids follow in later steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.hpp"

namespace pm {

pm_status graph_create(const pm_csr_view *csr, uint32_t flags, hipStream_t s, pm_graph **out);
void graph_free(pm_graph *g, hipStream_t s);
uint64_t graph_bytes_for(int64_t n, int64_t slots);
pm_status finalize(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t W,
                   uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta, pm_result *out);
pm_status samples_for_request(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t k0,
                              uint64_t W, uint64_t Lambda, uint64_t N1, uint32_t mask, double rel_err, double delta,
                              uint64_t k_max, uint64_t *k_path, uint64_t *k_cent, uint32_t *capped, uint32_t *unseen);
int sampler_cu_count(int dev);
std::string last_error_text();

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct SrvGraph {
    pm_csr_view csr{};
    uint32_t flags = 0;
    uint64_t est = 0;        // predicted resident bytes
    pm_graph *g = nullptr;   // resident prepared graph, or null
    uint64_t bytes = 0;      // its actual resident bytes
    int pins = 0;            // active requests on it
    uint64_t last_use = 0;   // LRU clock
    bool preparing = false;
    pm_status failed = PM_OK;  // sticky preparation error (invalid graph)
    std::string err;
};

struct SrvReq {
    uint64_t ticket = 0;
    pm_request rq{};
    int state = 0;           // 0 queued, 1 active, 2 done
    bool cancel = false;
    bool sized = false;      // final budgets known
    uint64_t k[2] = {0, 0};  // final budgets (reported)
    uint64_t next[2] = {0, 0};   // next id to issue
    uint64_t chunk[2] = {0, 0};  // ids in the step in flight
    uint64_t tally[2][PM_NUM_TALLIES] = {};
    int slot = -1;
    pm_status status = PM_OK;
    std::string err;
    pm_result result{};
    pm_req_stats st{};
    Clock::time_point t_submit, t_admit;
};

}  // namespace

}  // namespace pm

struct pm_server {
    int device = 0;
    pm_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_prep;
    std::mutex prep_mu;  // one preparation at a time (they share s_prep)
    std::vector<pm::SrvGraph> graphs;  // reserved to max_graphs: never moves
    std::deque<pm::SrvReq *> queue;
    std::vector<pm::SrvReq *> active;
    std::unordered_map<uint64_t, std::unique_ptr<pm::SrvReq>> reqs;
    std::vector<int> free_slots;
    uint64_t next_ticket = 1;
    uint64_t clock = 0;
    uint64_t resident = 0;  // bytes of resident graphs
    uint64_t reserved = 0;  // bytes of graphs being prepared
    bool stop = false;
    pm_server_stats stats{};
    std::thread worker;

    hipStream_t s_step = nullptr, s_prep = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    pm::BatchGraph *d_graphs = nullptr, *h_graphs = nullptr;  // h_ pinned
    pm::BatchTile *d_tiles = nullptr, *h_tiles = nullptr;
    uint32_t tile_cap = 0;
    pm::BatchCtl *d_ctl = nullptr, *h_ctl = nullptr;
    uint64_t *d_tallies = nullptr, *h_tallies = nullptr;
    unsigned max_blocks = 1;
};

namespace pm {

namespace {

bool graph_error(pm_status st) { return st == PM_EGRAPH || st == PM_EOVERFLOW || st == PM_EINVAL; }

// The target of the ids a sampler samples now: the pilot until sized, then
// the final budget; a sampler of zero weight samples nothing.
uint64_t target_of(const pm_server *S, const SrvReq *r, int tag)
{
    const pm_graph *g = S->graphs[r->rq.graph].g;
    const uint64_t R = tag == 0 ? g->R_tau : g->R_lam;
    if (R == 0) return 0;
    return r->sized ? r->k[tag] : S->cfg.k_pilot;
}

void finish(pm_server *S, SrvReq *r, pm_status st, const std::string &err)
{
    r->status = st;
    r->err = err;
    r->state = 2;
    r->st.latency_ms = ms_between(r->t_submit, Clock::now());
    if (r->slot >= 0) {
        S->free_slots.push_back(r->slot);
        r->slot = -1;
        SrvGraph &G = S->graphs[r->rq.graph];
        --G.pins;
        G.last_use = ++S->clock;
    }
    ++S->stats.requests_done;
    S->cv_done.notify_all();
}

// After a step (or at admission): size the budgets once the pilot is in,
// finalize once every id is in.
void advance(pm_server *S, SrvReq *r)
{
    const pm_graph *g = S->graphs[r->rq.graph].g;
    if (!r->sized && r->next[0] >= target_of(S, r, 0) && r->next[1] >= target_of(S, r, 1)) {
        uint64_t kp = 0, kc = 0;
        uint32_t capped = 0, unseen = 0;
        pm_status st = samples_for_request(r->tally[0], r->tally[1], S->cfg.k_pilot, g->R_tau / 2, g->R_lam / 2,
                                           g->N1, r->rq.motif_mask, r->rq.rel_err, r->rq.delta, S->cfg.k_max, &kp,
                                           &kc, &capped, &unseen);
        if (st != PM_OK) {
            finish(S, r, st, last_error_text());
            return;
        }
        r->k[0] = kp;
        r->k[1] = kc;
        r->st.capped_mask = capped;
        r->st.unseen_mask = unseen;
        r->sized = true;
    }
    if (r->sized && r->next[0] >= target_of(S, r, 0) && r->next[1] >= target_of(S, r, 1)) {
        pm_result out;
        pm_status st = finalize(r->tally[0], r->tally[1], g->R_tau / 2, g->R_lam / 2, g->N1, r->k[0], r->k[1],
                                r->rq.delta, &out);
        r->result = out;
        r->st.k_path = r->k[0];
        r->st.k_cent = r->k[1];
        finish(S, r, st, st == PM_OK ? std::string() : last_error_text());
    }
}

void evict(pm_server *S, SrvGraph &G)
{
    graph_free(G.g, S->s_prep);
    G.g = nullptr;
    S->resident -= G.bytes;
    G.bytes = 0;
    ++S->stats.evictions;
}

// Make graph gid resident; lk holds S->mu and is released while preparing.
// PM_EBUSY: it does not fit beside the pinned graphs now.
pm_status ensure_resident(pm_server *S, uint32_t gid, std::unique_lock<std::mutex> &lk, bool *prepared,
                          std::string *err)
{
    for (;;) {
        SrvGraph &G = S->graphs[gid];
        if (G.failed != PM_OK) {
            *err = G.err;
            return G.failed;
        }
        if (G.g) {
            G.last_use = ++S->clock;
            return PM_OK;
        }
        if (G.preparing) {
            S->cv_prep.wait(lk);
            continue;
        }
        if (G.est > S->cfg.hbm_budget) {
            *err = "graph needs " + std::to_string(G.est) + " bytes, more than the server's HBM budget";
            return PM_ENOMEM;
        }
        while (S->resident + S->reserved + G.est > S->cfg.hbm_budget) {
            SrvGraph *victim = nullptr;
            for (auto &H : S->graphs)
                if (H.g && H.pins == 0 && (!victim || H.last_use < victim->last_use)) victim = &H;
            if (!victim) break;
            evict(S, *victim);
        }
        if (S->resident + S->reserved + G.est > S->cfg.hbm_budget) {
            *err = "graph does not fit beside the graphs in use";
            return PM_EBUSY;
        }
        G.preparing = true;
        S->reserved += G.est;
        const pm_csr_view csr = G.csr;
        const uint32_t flags = G.flags;
        lk.unlock();
        pm_graph *g = nullptr;
        pm_status st;
        std::string msg;
        {
            std::lock_guard<std::mutex> pl(S->prep_mu);
            st = graph_create(&csr, flags, S->s_prep, &g);
            if (st == PM_OK) {
                BatchGraph &d = S->h_graphs[gid];
                d.v[0] = view_of(g, false);
                d.v[1] = view_of(g, true);
                hipError_t e = hipMemcpyAsync(S->d_graphs + gid, &d, sizeof(BatchGraph), hipMemcpyHostToDevice,
                                              S->s_prep);
                if (e == hipSuccess) e = hipStreamSynchronize(S->s_prep);
                if (e != hipSuccess) {
                    st = PM_EDEVICE;
                    set_error(std::string("server: descriptor upload: ") + hipGetErrorString(e));
                }
            }
            if (st != PM_OK) msg = last_error_text();
            if (st != PM_OK && g) {
                graph_free(g, S->s_prep);
                g = nullptr;
            }
        }
        lk.lock();
        G.preparing = false;
        S->reserved -= G.est;
        S->cv_prep.notify_all();
        if (st != PM_OK) {
            if (graph_error(st)) {
                G.failed = st;
                G.err = msg;
            }
            *err = msg;
            return st;
        }
        G.g = g;
        G.bytes = g->bytes;
        G.last_use = ++S->clock;
        S->resident += G.bytes;
        ++S->stats.preparations;
        if (prepared) *prepared = true;
        return PM_OK;
    }
}

// Admit queued requests in order while slots are free and their graphs fit.
void admit(pm_server *S, std::unique_lock<std::mutex> &lk)
{
    while (!S->queue.empty() && !S->free_slots.empty()) {
        SrvReq *r = S->queue.front();
        if (r->cancel) {
            S->queue.pop_front();
            finish(S, r, PM_ECANCELED, "request cancelled");
            continue;
        }
        bool prepared = false;
        std::string err;
        pm_status st = ensure_resident(S, r->rq.graph, lk, &prepared, &err);
        if (st == PM_EBUSY) return;  // first come, first served: wait for memory
        // the lock was dropped: the queue head is still r (only this thread pops)
        S->queue.pop_front();
        if (st != PM_OK) {
            finish(S, r, st, err);
            continue;
        }
        if (r->cancel) {
            finish(S, r, PM_ECANCELED, "request cancelled");
            continue;
        }
        r->slot = S->free_slots.back();
        S->free_slots.pop_back();
        ++S->graphs[r->rq.graph].pins;
        r->state = 1;
        r->st.prepared = prepared ? 1 : 0;
        r->t_admit = Clock::now();
        r->st.queued_ms = ms_between(r->t_submit, r->t_admit);
        S->active.push_back(r);
        advance(S, r);  // nothing to sample (zero weights): done at once
        if (r->state == 2) S->active.pop_back();
    }
}

pm_status grow_tiles(pm_server *S, uint32_t need)
{
    if (need <= S->tile_cap) return PM_OK;
    uint32_t cap = std::max<uint32_t>(need, S->tile_cap * 2);
    dev_free(S->d_tiles, S->s_step);
    if (S->h_tiles) (void)hipHostFree(S->h_tiles);
    S->d_tiles = nullptr;
    S->h_tiles = nullptr;
    S->tile_cap = 0;
    PM_TRY(dev_alloc((void **)&S->d_tiles, sizeof(BatchTile) * cap, S->s_step));
    PM_HIP(hipHostMalloc((void **)&S->h_tiles, sizeof(BatchTile) * cap, hipHostMallocDefault));
    S->tile_cap = cap;
    return PM_OK;
}

// Cut this step's chunks: the pilot whole, otherwise an equal share of
// step_samples per (request, sampler) with work left, in whole tiles.
pm_status build_step(pm_server *S, uint32_t *ntiles)
{
    const uint64_t tile = (uint64_t)S->cfg.samples_per_tile;
    uint64_t nwork = 0;
    for (SrvReq *r : S->active)
        for (int tag = 0; tag < 2; ++tag)
            if (r->next[tag] < target_of(S, r, tag)) ++nwork;
    uint64_t share = S->cfg.step_samples / std::max<uint64_t>(nwork, 1);
    share = std::max<uint64_t>(tile, (share + tile - 1) / tile * tile);
    uint64_t need = 0;
    for (SrvReq *r : S->active)
        for (int tag = 0; tag < 2; ++tag) {
            const uint64_t rem = target_of(S, r, tag) - std::min(r->next[tag], target_of(S, r, tag));
            r->chunk[tag] = r->sized ? std::min(rem, share) : rem;
            need += (r->chunk[tag] + tile - 1) / tile;
        }
    if (need > 0xFFFFFFF0ull) {
        set_error("server: step too large");
        return PM_EINVAL;
    }
    PM_TRY(grow_tiles(S, (uint32_t)need));
    uint32_t n = 0;
    for (SrvReq *r : S->active)
        for (int tag = 0; tag < 2; ++tag)
            for (uint64_t done = 0; done < r->chunk[tag]; done += tile) {
                BatchTile &t = S->h_tiles[n++];
                t.graph = r->rq.graph;
                t.tag = (uint32_t)tag;
                t.count = (uint32_t)std::min<uint64_t>(tile, r->chunk[tag] - done);
                t.slot = (uint32_t)r->slot;
                t.first = r->next[tag] + done;
                t.seed = r->rq.seed;
            }
    *ntiles = n;
    return PM_OK;
}

pm_status launch_step(pm_server *S, uint32_t ntiles)
{
    S->h_ctl->ntiles = ntiles;
    S->h_ctl->cursor = 0;
    S->h_ctl->nlists = 0;  // one cursor
    const size_t tb = sizeof(uint64_t) * (size_t)S->cfg.max_active * 2 * PM_NUM_TALLIES;
    PM_HIP(hipEventRecord(S->ev_a, S->s_step));
    PM_HIP(hipMemcpyAsync(S->d_tiles, S->h_tiles, sizeof(BatchTile) * ntiles, hipMemcpyHostToDevice, S->s_step));
    PM_HIP(hipMemcpyAsync(S->d_ctl, S->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, S->s_step));
    PM_TRY(fill_async<uint64_t>(S->d_tallies, 0ull, (int64_t)S->cfg.max_active * 2 * PM_NUM_TALLIES, S->s_step));
    const unsigned blocks = (unsigned)std::max<uint32_t>(1, std::min<uint32_t>(S->max_blocks, ntiles));
    PM_TRY(launch_tiles(S->d_graphs, S->d_tiles, S->d_ctl, S->d_tallies, blocks, S->s_step));
    PM_HIP(hipMemcpyAsync(S->h_tallies, S->d_tallies, tb, hipMemcpyDeviceToHost, S->s_step));
    PM_HIP(hipEventRecord(S->ev_b, S->s_step));
    return PM_OK;
}

void fail_active(pm_server *S, pm_status st, const std::string &err)
{
    for (SrvReq *r : S->active) finish(S, r, st, err);
    S->active.clear();
}

void worker_main(pm_server *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [S] { return S->stop || !S->queue.empty() || !S->active.empty(); });
        if (S->stop) {
            for (SrvReq *r : S->queue) finish(S, r, PM_ECANCELED, "server destroyed");
            S->queue.clear();
            fail_active(S, PM_ECANCELED, "server destroyed");
            return;
        }
        // drop cancelled active requests
        for (size_t i = 0; i < S->active.size();) {
            SrvReq *r = S->active[i];
            if (r->cancel) {
                finish(S, r, PM_ECANCELED, "request cancelled");
                S->active[i] = S->active.back();
                S->active.pop_back();
            } else {
                ++i;
            }
        }
        bool launched = false;
        if (!S->active.empty()) {
            uint32_t ntiles = 0;
            pm_status st = build_step(S, &ntiles);
            if (st == PM_OK && ntiles > 0) st = launch_step(S, ntiles);
            if (st != PM_OK) {
                fail_active(S, st, last_error_text());
            } else {
                launched = ntiles > 0;
            }
        }
        // admissions (and graph preparations) overlap the step in flight
        const size_t before = S->active.size();
        admit(S, lk);
        if (!launched) {
            if (S->active.size() == before && !S->queue.empty() && S->active.empty()) {
                // head of the queue waits for memory that nothing running will free
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
            continue;
        }
        lk.unlock();
        hipError_t e = hipEventSynchronize(S->ev_b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, S->ev_a, S->ev_b);
        lk.lock();
        if (e != hipSuccess) {
            fail_active(S, PM_EDEVICE, std::string("server step: ") + hipGetErrorString(e));
            continue;
        }
        ++S->stats.steps;
        S->stats.busy_ms += ms;
        std::vector<SrvReq *> still;
        still.reserve(S->active.size());
        for (SrvReq *r : S->active) {
            if (r->state != 1) continue;
            const bool had = r->chunk[0] + r->chunk[1] > 0;
            if (had) {
                const uint64_t *t = S->h_tallies + (size_t)r->slot * 2 * PM_NUM_TALLIES;
                for (int tag = 0; tag < 2; ++tag) {
                    for (int c = 0; c < PM_NUM_TALLIES; ++c) r->tally[tag][c] += t[tag * PM_NUM_TALLIES + c];
                    r->next[tag] += r->chunk[tag];
                    S->stats.samples += r->chunk[tag];
                    r->chunk[tag] = 0;
                }
                ++r->st.steps;
            }
            advance(S, r);
            if (r->state == 1) still.push_back(r);
        }
        S->active.swap(still);
    }
}

pm_status check_request(const pm_server *S, const pm_request *q)
{
    if (q->graph >= S->graphs.size()) {
        set_error("server: unknown graph id");
        return PM_EINVAL;
    }
    if (!(q->delta > 0.0 && q->delta < 1.0)) {
        set_error("server: delta must lie in (0,1)");
        return PM_EINVAL;
    }
    const bool fixed = q->k_path != 0 || q->k_cent != 0;
    if (!fixed && !(q->rel_err > 0.0 && q->rel_err < 1.0)) {
        set_error("server: rel_err must lie in (0,1) when the budgets are sized");
        return PM_EINVAL;
    }
    if (q->motif_mask & ~0x7eu) {
        set_error("server: motif_mask has bits outside 1..6");
        return PM_EINVAL;
    }
    return PM_OK;
}

void server_free(pm_server *S)
{
    if (S->s_step) (void)hipStreamSynchronize(S->s_step);
    if (S->s_prep) (void)hipStreamSynchronize(S->s_prep);
    for (auto &G : S->graphs)
        if (G.g) graph_free(G.g, S->s_prep);
    dev_free(S->d_graphs, S->s_step);
    dev_free(S->d_tiles, S->s_step);
    dev_free(S->d_ctl, S->s_step);
    dev_free(S->d_tallies, S->s_step);
    if (S->h_graphs) (void)hipHostFree(S->h_graphs);
    if (S->h_tiles) (void)hipHostFree(S->h_tiles);
    if (S->h_ctl) (void)hipHostFree(S->h_ctl);
    if (S->h_tallies) (void)hipHostFree(S->h_tallies);
    if (S->ev_a) (void)hipEventDestroy(S->ev_a);
    if (S->ev_b) (void)hipEventDestroy(S->ev_b);
    if (S->s_step) {
        (void)hipStreamSynchronize(S->s_step);
        (void)hipStreamDestroy(S->s_step);
    }
    if (S->s_prep) {
        (void)hipStreamSynchronize(S->s_prep);
        (void)hipStreamDestroy(S->s_prep);
    }
    delete S;
}

}  // namespace

pm_status server_create(const pm_server_cfg *cfg_in, pm_server **out)
{
    if (!out) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    *out = nullptr;
    pm_server_cfg c{};
    if (cfg_in) c = *cfg_in;
    if (c.max_active < 0 || c.max_graphs < 0 || c.samples_per_tile < 0 || c.blocks_per_cu < 0 ||
        c.blocks_per_cu > 64 || (c.samples_per_tile > 0 && c.samples_per_tile < 64)) {
        set_error("server: negative limit, samples_per_tile below 64 or blocks_per_cu above 64");
        return PM_EINVAL;
    }
    if (c.max_active == 0) c.max_active = 256;
    if (c.max_graphs == 0) c.max_graphs = 1024;
    if (c.step_samples == 0) c.step_samples = 1ull << 25;
    if (c.k_pilot == 0) c.k_pilot = 65536;
    if (c.k_max == 0) c.k_max = 2000000000ull;
    if (c.samples_per_tile == 0) c.samples_per_tile = 4096;
    if (c.blocks_per_cu == 0) c.blocks_per_cu = 4;
    if (c.k_max < c.k_pilot) {
        set_error("server: k_max below k_pilot");
        return PM_EINVAL;
    }
    pm_server *S = new (std::nothrow) pm_server();
    if (!S) return PM_ENOMEM;
    struct Guard {
        pm_server *s;
        ~Guard()
        {
            if (s) server_free(s);
        }
    } guard{S};
    PM_HIP(hipGetDevice(&S->device));
    if (c.hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        PM_HIP(hipMemGetInfo(&free_b, &total_b));
        c.hbm_budget = free_b / 4 * 3;
    }
    S->cfg = c;
    S->graphs.reserve((size_t)c.max_graphs);
    for (int i = c.max_active - 1; i >= 0; --i) S->free_slots.push_back(i);
    PM_HIP(hipStreamCreateWithFlags(&S->s_step, hipStreamNonBlocking));
    PM_HIP(hipStreamCreateWithFlags(&S->s_prep, hipStreamNonBlocking));
    PM_HIP(hipEventCreate(&S->ev_a));
    PM_HIP(hipEventCreate(&S->ev_b));
    PM_TRY(dev_alloc((void **)&S->d_graphs, sizeof(BatchGraph) * c.max_graphs, S->s_step));
    PM_HIP(hipHostMalloc((void **)&S->h_graphs, sizeof(BatchGraph) * c.max_graphs, hipHostMallocDefault));
    std::memset((void *)S->h_graphs, 0, sizeof(BatchGraph) * c.max_graphs);
    PM_TRY(dev_alloc((void **)&S->d_ctl, sizeof(BatchCtl), S->s_step));
    PM_HIP(hipHostMalloc((void **)&S->h_ctl, sizeof(BatchCtl), hipHostMallocDefault));
    const size_t tb = sizeof(uint64_t) * (size_t)c.max_active * 2 * PM_NUM_TALLIES;
    PM_TRY(dev_alloc((void **)&S->d_tallies, tb, S->s_step));
    PM_HIP(hipHostMalloc((void **)&S->h_tallies, tb, hipHostMallocDefault));
    PM_TRY(grow_tiles(S, (uint32_t)std::min<uint64_t>(1u << 20, c.step_samples / c.samples_per_tile + 2 * c.max_active)));
    PM_HIP(hipStreamSynchronize(S->s_step));
    S->max_blocks = (unsigned)std::max(1, sampler_cu_count(S->device) * c.blocks_per_cu);
    S->worker = std::thread(worker_main, S);
    guard.s = nullptr;
    *out = S;
    return PM_OK;
}

pm_status server_add_graph(pm_server *S, const pm_csr_view *csr, uint32_t flags, uint32_t *gid)
{
    if (!S || !csr || !gid || !csr->row_offsets || csr->n < 0 || csr->n > (int64_t)INT32_MAX) {
        set_error("server: null argument or n outside [0, 2^31)");
        return PM_EINVAL;
    }
    int64_t slots = 0;
    if (csr->on_device) {
        int dev = 0;
        PM_HIP(hipGetDevice(&dev));
        PM_HIP(hipSetDevice(S->device));
        hipError_t e = hipMemcpy(&slots, csr->row_offsets + csr->n, sizeof(int64_t), hipMemcpyDeviceToHost);
        (void)hipSetDevice(dev);
        PM_HIP(e);
    } else {
        slots = csr->row_offsets[csr->n];
    }
    if (slots < 0) slots = 0;  // an invalid graph fails at preparation
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->graphs.size() >= (size_t)S->cfg.max_graphs) {
        set_error("server: max_graphs reached");
        return PM_EINVAL;
    }
    SrvGraph G;
    G.csr = *csr;
    G.flags = flags;
    G.est = graph_bytes_for(csr->n, slots);
    S->graphs.push_back(G);
    *gid = (uint32_t)(S->graphs.size() - 1);
    return PM_OK;
}

pm_status server_preload(pm_server *S, uint32_t gid)
{
    if (!S) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    int dev = 0;
    PM_HIP(hipGetDevice(&dev));
    PM_HIP(hipSetDevice(S->device));
    std::unique_lock<std::mutex> lk(S->mu);
    pm_status st;
    std::string err;
    if (gid >= S->graphs.size()) {
        err = "server: unknown graph id";
        st = PM_EINVAL;
    } else {
        st = ensure_resident(S, gid, lk, nullptr, &err);
    }
    lk.unlock();
    (void)hipSetDevice(dev);
    if (st != PM_OK) set_error(err);
    return st;
}

pm_status server_submit(pm_server *S, const pm_request *q, uint64_t *ticket)
{
    if (!S || !q || !ticket) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    PM_TRY(check_request(S, q));
    if (S->stop) {
        set_error("server: shutting down");
        return PM_ECANCELED;
    }
    std::unique_ptr<SrvReq> r(new SrvReq());
    r->ticket = S->next_ticket++;
    r->rq = *q;
    r->t_submit = Clock::now();
    if (q->k_path != 0 || q->k_cent != 0) {
        r->sized = true;
        r->k[0] = q->k_path;
        r->k[1] = q->k_cent;
    }
    S->queue.push_back(r.get());
    *ticket = r->ticket;
    S->reqs.emplace(r->ticket, std::move(r));
    S->cv_work.notify_one();
    return PM_OK;
}

pm_status server_wait(pm_server *S, uint64_t ticket, int64_t timeout_ms, pm_result *out, pm_req_stats *st)
{
    if (!S) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("server: unknown ticket");
        return PM_EINVAL;
    }
    SrvReq *r = it->second.get();
    auto done = [r] { return r->state == 2; };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, done);
    } else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        set_error("server: wait timed out");
        return PM_EBUSY;
    }
    const pm_status status = r->status;
    if (out) *out = r->result;
    if (st) *st = r->st;
    if (status != PM_OK) set_error(r->err);
    S->reqs.erase(it);
    return status;
}

pm_status server_cancel(pm_server *S, uint64_t ticket)
{
    if (!S) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("server: unknown ticket");
        return PM_EINVAL;
    }
    it->second->cancel = true;
    S->cv_work.notify_one();
    return PM_OK;
}

pm_status server_get_stats(pm_server *S, pm_server_stats *out)
{
    if (!S || !out) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->resident_bytes = S->resident;
    uint64_t n = 0;
    for (auto &G : S->graphs) n += G.g != nullptr;
    out->resident_graphs = n;
    return PM_OK;
}

pm_status server_destroy(pm_server *S)
{
    if (!S) {
        set_error("server: null argument");
        return PM_EINVAL;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    server_free(S);
    return PM_OK;
}

}  // namespace pm
