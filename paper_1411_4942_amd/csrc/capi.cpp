// The C ABI of include/pathsamp.h: argument checks, error strings, and the
// one-shot and prepared-graph entry points.  No exception leaves this file.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "../../include/pathsamp.h"

struct pm_graph;

namespace pm {

static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }
std::string last_error_text() { return t_last_error; }

pm_status graph_create(const pm_csr_view *csr, uint32_t flags, hipStream_t s, pm_graph **out);
void graph_free(pm_graph *g, hipStream_t s);
pm_status graph_export(const pm_graph *g, int64_t *off, int32_t *col, int32_t *rank, uint64_t *p_tau,
                       uint64_t *p_lam, hipStream_t s);
pm_status graph_info(const pm_graph *g, pm_graph_info *out);
pm_status sample_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, hipStream_t s);
pm_status graph_build_alias(pm_graph *g, hipStream_t s);
pm_status graph_alias_export(const pm_graph *g, int32_t centered, uint64_t *K, int64_t *alias, hipStream_t s);
pm_status count_alias(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s);
pm_status finalize(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t W,
                   uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta, pm_result *out);
pm_status chernoff_interval(uint64_t count, uint64_t k, double delta, double *p_lo, double *p_hi);
pm_status samples_for_error(double rel_err, double delta, double alpha, uint64_t *k_out);
pm_status philox_device(const uint32_t *in, uint32_t *out, int64_t count);
pm_status device_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s);
pm_status device_gather(const void *table, uint64_t bytes, int64_t count, uint64_t seed, hipStream_t s);
pm_status dev_alloc(void **p, size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
pm_status count_on_graph(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s);
pm_status set_sampler_shape(int32_t samples_per_lane, int32_t blocks_per_cu);
pm_status set_draw_order(int32_t enabled, uint64_t min_samples);
pm_status set_search_mode(int32_t mode);
pm_status count_noalloc(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s);
size_t static_scratch_bytes();
pm_status adjacent(const pm_graph *g, const int32_t *a, const int32_t *b, int64_t count, uint8_t *out, int32_t mode,
                   hipStream_t s);
pm_status draw_order(const pm_graph *g, int32_t centered, uint64_t seed, uint64_t first, uint64_t k, uint32_t *out,
                     hipStream_t s);
pm_status batch_create(const pm_graph *const *graphs, const pm_params *params, int32_t count, const pm_tune *tune,
                       hipStream_t user_stream, pm_batch **out);
pm_status batch_set_params(pm_batch *b, const pm_params *params);
pm_status batch_run(pm_batch *b, pm_result *out, hipStream_t user_stream);
pm_status batch_get_tune(const pm_batch *b, pm_tune *out);
pm_status batch_destroy(pm_batch *b);
pm_status csr_from_edges(const pm_edge_view *ev, int64_t *off, int32_t *col, int64_t capacity, int64_t *slots_out,
                         hipStream_t s);
pm_status graph_from_edges(const pm_edge_view *ev, uint32_t flags, hipStream_t s, pm_graph **out);
pm_status exact_counts(const pm_graph *g, pm_exact *out, hipStream_t s);
pm_status samples_for_request(const uint64_t tp[PM_NUM_TALLIES], const uint64_t tc[PM_NUM_TALLIES], uint64_t k0,
                              uint64_t W, uint64_t Lambda, uint64_t N1, uint32_t mask, double rel_err, double delta,
                              uint64_t k_max, uint64_t *k_path, uint64_t *k_cent, uint32_t *capped, uint32_t *unseen);
pm_status server_create(const pm_server_cfg *cfg, pm_server **out);
pm_status server_add_graph(pm_server *S, const pm_csr_view *csr, uint32_t flags, uint32_t *gid);
pm_status server_preload(pm_server *S, uint32_t gid);
pm_status server_submit(pm_server *S, const pm_request *q, uint64_t *ticket);
pm_status server_wait(pm_server *S, uint64_t ticket, int64_t timeout_ms, pm_result *out, pm_req_stats *st);
pm_status server_cancel(pm_server *S, uint64_t ticket);
pm_status server_get_stats(pm_server *S, pm_server_stats *out);
pm_status server_destroy(pm_server *S);

}  // namespace pm

#define PM_GUARD(body)                                          \
    try {                                                       \
        body                                                    \
    } catch (const std::bad_alloc &) {                          \
        pm::set_error("host allocation failed");                \
        return PM_ENOMEM;                                       \
    } catch (...) {                                             \
        pm::set_error("unexpected internal error");             \
        return PM_EDEVICE;                                      \
    }

extern "C" {

const char *pm_status_string(pm_status s)
{
    switch (s) {
    case PM_OK: return "PM_OK";
    case PM_EINVAL: return "PM_EINVAL";
    case PM_EGRAPH: return "PM_EGRAPH";
    case PM_EOVERFLOW: return "PM_EOVERFLOW";
    case PM_ENOMEM: return "PM_ENOMEM";
    case PM_EDEVICE: return "PM_EDEVICE";
    case PM_EBUSY: return "PM_EBUSY";
    case PM_ECANCELED: return "PM_ECANCELED";
    default: return "PM_UNKNOWN";
    }
}

const char *pm_last_error(void) { return pm::t_last_error.c_str(); }

pm_status pm_graph_create(const pm_csr_view *csr, uint32_t flags, void *stream, pm_graph **out)
{
    PM_GUARD(return pm::graph_create(csr, flags, (hipStream_t)stream, out);)
}

pm_status pm_graph_destroy(pm_graph *g)
{
    PM_GUARD({
        if (!g) {
            pm::set_error("null graph");
            return PM_EINVAL;
        }
        // samplers may still read the graph on a caller's stream
        // (pm_sample_async): wait for the whole device before freeing
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            pm::set_error(std::string("pm_graph_destroy: ") + hipGetErrorString(e));
            return PM_EDEVICE;
        }
        pm::graph_free(g, nullptr);
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            pm::set_error(std::string("pm_graph_destroy: ") + hipGetErrorString(e));
            return PM_EDEVICE;
        }
        return PM_OK;
    })
}

pm_status pm_graph_info_get(const pm_graph *g, pm_graph_info *out)
{
    PM_GUARD(return pm::graph_info(g, out);)
}

pm_status pm_graph_export(const pm_graph *g, int64_t *off, int32_t *col, int32_t *rank, uint64_t *p_tau,
                          uint64_t *p_lam, void *stream)
{
    PM_GUARD(return pm::graph_export(g, off, col, rank, p_tau, p_lam, (hipStream_t)stream);)
}

pm_status pm_sample_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, void *stream)
{
    PM_GUARD(return pm::sample_async(g, p, tallies_dev, (hipStream_t)stream);)
}

pm_status pm_count(const pm_graph *g, const pm_params *p, pm_result *out, void *stream)
{
    PM_GUARD(return pm::count_on_graph(g, p, out, (hipStream_t)stream);)
}

pm_status pm_count_noalloc(const pm_graph *g, const pm_params *p, pm_result *out, void *stream)
{
    PM_GUARD(return pm::count_noalloc(g, p, out, (hipStream_t)stream);)
}

uint64_t pm_static_scratch_bytes(void) { return (uint64_t)pm::static_scratch_bytes(); }

pm_status pm_graph_build_alias(pm_graph *g, void *stream)
{
    PM_GUARD(return pm::graph_build_alias(g, (hipStream_t)stream);)
}

pm_status pm_count_alias(const pm_graph *g, const pm_params *p, pm_result *out, void *stream)
{
    PM_GUARD(return pm::count_alias(g, p, out, (hipStream_t)stream);)
}

pm_status pm_graph_alias_export(const pm_graph *g, int32_t centered, uint64_t *K, int64_t *alias, void *stream)
{
    PM_GUARD(return pm::graph_alias_export(g, centered, K, alias, (hipStream_t)stream);)
}

pm_status pm_count_motifs(const pm_csr_view *csr, uint64_t k, uint64_t seed, pm_result *out)
{
    PM_GUARD({
        if (!csr || !out || k == 0) {
            pm::set_error("pm_count_motifs: null argument or k == 0");
            return PM_EINVAL;
        }
        pm_graph *g = nullptr;
        pm_status st = pm::graph_create(csr, PM_VALIDATE | PM_CHECK_SYMMETRY, nullptr, &g);
        if (st != PM_OK) return st;
        pm_params p;
        std::memset(&p, 0, sizeof(p));
        p.k_path = k;
        p.k_cent = k;
        p.seed = seed;
        p.delta = 0.01;
        st = pm::count_on_graph(g, &p, out, nullptr);
        // samplers may still read the graph on a caller's stream
        // (pm_sample_async): wait for the whole device before freeing
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            pm::set_error(std::string("pm_graph_destroy: ") + hipGetErrorString(e));
            return PM_EDEVICE;
        }
        pm::graph_free(g, nullptr);
        e = hipStreamSynchronize(nullptr);
        if (st == PM_OK && e != hipSuccess) {
            pm::set_error(std::string("pm_count_motifs: ") + hipGetErrorString(e));
            return PM_EDEVICE;
        }
        return st;
    })
}

pm_status pm_finalize(const uint64_t tally_path[PM_NUM_TALLIES], const uint64_t tally_cent[PM_NUM_TALLIES],
                      uint64_t W, uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta,
                      pm_result *out)
{
    PM_GUARD(return pm::finalize(tally_path, tally_cent, W, Lambda, N1, k_path, k_cent, delta, out);)
}

pm_status pm_chernoff_interval(uint64_t count, uint64_t k, double delta, double *p_lo, double *p_hi)
{
    PM_GUARD(return pm::chernoff_interval(count, k, delta, p_lo, p_hi);)
}

pm_status pm_exact_counts(const pm_graph *g, pm_exact *out, void *stream)
{
    PM_GUARD(return pm::exact_counts(g, out, (hipStream_t)stream);)
}

pm_status pm_csr_from_edges(const pm_edge_view *edges, int64_t *off, int32_t *col, int64_t capacity,
                            int64_t *slots_out, void *stream)
{
    PM_GUARD(return pm::csr_from_edges(edges, off, col, capacity, slots_out, (hipStream_t)stream);)
}

pm_status pm_graph_from_edges(const pm_edge_view *edges, uint32_t flags, void *stream, pm_graph **out)
{
    PM_GUARD(return pm::graph_from_edges(edges, flags, (hipStream_t)stream, out);)
}

pm_status pm_samples_for_error(double rel_err, double delta, double alpha, uint64_t *k_out)
{
    PM_GUARD(return pm::samples_for_error(rel_err, delta, alpha, k_out);)
}

pm_status pm_samples_for_request(const uint64_t tally_path[PM_NUM_TALLIES], const uint64_t tally_cent[PM_NUM_TALLIES],
                                 uint64_t k0, uint64_t W, uint64_t Lambda, uint64_t N1, uint32_t motif_mask,
                                 double rel_err, double delta, uint64_t k_max, uint64_t *k_path, uint64_t *k_cent,
                                 uint32_t *capped, uint32_t *unseen)
{
    PM_GUARD(return pm::samples_for_request(tally_path, tally_cent, k0, W, Lambda, N1, motif_mask, rel_err, delta,
                                            k_max, k_path, k_cent, capped, unseen);)
}

pm_status pm_server_create(const pm_server_cfg *cfg, pm_server **out)
{
    PM_GUARD(return pm::server_create(cfg, out);)
}

pm_status pm_server_add_graph(pm_server *srv, const pm_csr_view *csr, uint32_t flags, uint32_t *graph_id)
{
    PM_GUARD(return pm::server_add_graph(srv, csr, flags, graph_id);)
}

pm_status pm_server_preload(pm_server *srv, uint32_t graph_id)
{
    PM_GUARD(return pm::server_preload(srv, graph_id);)
}

pm_status pm_server_submit(pm_server *srv, const pm_request *req, uint64_t *ticket)
{
    PM_GUARD(return pm::server_submit(srv, req, ticket);)
}

pm_status pm_server_wait(pm_server *srv, uint64_t ticket, int64_t timeout_ms, pm_result *out, pm_req_stats *st)
{
    PM_GUARD(return pm::server_wait(srv, ticket, timeout_ms, out, st);)
}

pm_status pm_server_cancel(pm_server *srv, uint64_t ticket)
{
    PM_GUARD(return pm::server_cancel(srv, ticket);)
}

pm_status pm_server_get_stats(pm_server *srv, pm_server_stats *out)
{
    PM_GUARD(return pm::server_get_stats(srv, out);)
}

pm_status pm_server_destroy(pm_server *srv)
{
    PM_GUARD(return pm::server_destroy(srv);)
}

pm_status pm_set_sampler_shape(int32_t samples_per_lane, int32_t blocks_per_cu)
{
    PM_GUARD(return pm::set_sampler_shape(samples_per_lane, blocks_per_cu);)
}

pm_status pm_set_draw_order(int32_t enabled, uint64_t min_samples)
{
    PM_GUARD(return pm::set_draw_order(enabled, min_samples);)
}

pm_status pm_set_search_mode(int32_t mode)
{
    PM_GUARD(return pm::set_search_mode(mode);)
}

pm_status pm_batch_create(const pm_graph *const *graphs, const pm_params *params, int32_t count, const pm_tune *tune,
                          void *stream, pm_batch **out)
{
    PM_GUARD(return pm::batch_create(graphs, params, count, tune, (hipStream_t)stream, out);)
}

pm_status pm_batch_set_params(pm_batch *b, const pm_params *params)
{
    PM_GUARD(return pm::batch_set_params(b, params);)
}

pm_status pm_batch_run(pm_batch *b, pm_result *out, void *stream)
{
    PM_GUARD(return pm::batch_run(b, out, (hipStream_t)stream);)
}

pm_status pm_batch_get_tune(const pm_batch *b, pm_tune *out)
{
    PM_GUARD(return pm::batch_get_tune(b, out);)
}

pm_status pm_batch_destroy(pm_batch *b)
{
    PM_GUARD(return pm::batch_destroy(b);)
}

pm_status pm_count_batch(const pm_graph *const *graphs, const pm_params *params, pm_result *out, int32_t count,
                         const pm_tune *tune, void *stream)
{
    PM_GUARD({
        pm_batch *b = nullptr;
        pm_status st = pm::batch_create(graphs, params, count, tune, (hipStream_t)stream, &b);
        if (st != PM_OK) return st;
        st = pm::batch_run(b, out, (hipStream_t)stream);
        pm::batch_destroy(b);
        return st;
    })
}

pm_status pm_device_copy(void *dst, const void *src, uint64_t bytes, void *stream)
{
    PM_GUARD(return pm::device_copy(dst, src, bytes, (hipStream_t)stream);)
}

pm_status pm_device_gather(const void *table, uint64_t bytes, int64_t count, uint64_t seed, void *stream)
{
    PM_GUARD(return pm::device_gather(table, bytes, count, seed, (hipStream_t)stream);)
}

pm_status pm_adjacent(const pm_graph *g, const int32_t *a, const int32_t *b, int64_t count, uint8_t *out,
                      int32_t mode, void *stream)
{
    PM_GUARD(return pm::adjacent(g, a, b, count, out, mode, (hipStream_t)stream);)
}

pm_status pm_draw_order(const pm_graph *g, int32_t centered, uint64_t seed, uint64_t first_id, uint64_t k,
                        uint32_t *ids_out, void *stream)
{
    PM_GUARD(return pm::draw_order(g, centered, seed, first_id, k, ids_out, (hipStream_t)stream);)
}

pm_status pm_philox_device(const uint32_t *in, uint32_t *out, int64_t count)
{
    PM_GUARD(return pm::philox_device(in, out, count);)
}

}  // extern "C"
