/*
 * pathsamp -- 3-path sampling for the six connected 4-vertex induced subgraph
 * counts (Jha, Seshadhri, Pinar, "Path Sampling: A Fast and Provable Method
 * for Estimating 4-Vertex Subgraph Counts"), as HIP kernels for MI355X
 * (gfx950) behind a C ABI.
 *
 * Motif numbering (the paper's Figure 1): 1 3-star, 2 3-path,
 * 3 tailed-triangle, 4 4-cycle, 5 chordal-4-cycle, 6 4-clique.
 *
 * Conventions for every call:
 *  - Every function returns a pm_status: PM_OK (0) or a negative code.  On
 *    failure pm_last_error() holds a message for the calling thread.
 *  - "stream" arguments are hipStream_t values passed as void*; NULL means
 *    the default stream.  Calls that take a stream return after the results
 *    they report are on the host (they synchronise that stream).
 *  - A call may run part of its work on the library's own side streams (two
 *    per device, default priority): they wait for the work already on
 *    `stream`, and `stream` waits for them before anything the call enqueues
 *    after them, so everything the call does is ordered on `stream` as if it
 *    ran there (pm_sample_async's tallies are complete once `stream` has
 *    passed the call).
 *  - The caller owns every buffer it passes in; the library never frees or
 *    keeps a pointer to caller memory past the call.
 *  - No C++ exception crosses this boundary.
 */
#ifndef PATHSAMP_H
#define PATHSAMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pm_status;

#define PM_OK 0
#define PM_EINVAL (-1)     /* null pointer, n < 0, k == 0, delta outside (0,1), size limit */
#define PM_EGRAPH (-2)     /* CSR not an undirected simple graph (see pm_graph_create) */
#define PM_EOVERFLOW (-3)  /* 2W, 2 Lambda or N_1 does not fit in 64 bits */
#define PM_ENOMEM (-4)     /* device or host allocation failed */
#define PM_EDEVICE (-5)    /* a HIP runtime call failed */
#define PM_EBUSY (-6)      /* server: request does not fit the memory budget now */
#define PM_ECANCELED (-7)  /* server: request cancelled */

/* Tally slots.  3-path sampler: TRI (u' = v'), then motifs 2..6.
 * Centered sampler: TRI (u' = v'), OPEN (not a centered 3-path), motifs 4..6. */
#define PM_TALLY_TRI 0
#define PM_TALLY_OPEN 1
#define PM_NUM_TALLIES 8

/* Flags of pm_graph_create. */
#define PM_VALIDATE 1u        /* check offsets, ranges, self-loops, sorted rows */
#define PM_CHECK_SYMMETRY 2u  /* also check that every edge appears in both rows */

/* An input graph in CSR form.  row_offsets has n+1 entries, starting at 0
 * and non-decreasing; cols has row_offsets[n] entries, each row strictly
 * ascending.  The graph must be undirected (every edge stored in both rows)
 * and simple (no self-loops, no repeated edge): the input of Section 2.
 * on_device != 0 means both pointers are device memory of the current HIP
 * device; otherwise they are host memory and are copied in. */
typedef struct {
    int64_t n;
    const int64_t *row_offsets;
    const int32_t *cols;
    int32_t on_device;
} pm_csr_view;

/* Sampling parameters.  k_path samples of Algorithm 2 (3-path-sampler) and
 * k_cent of Algorithm 4 (centered-sampler); sample ids first_id ..
 * first_id + k - 1 of each sampler, so disjoint id ranges of one seed add up
 * to one longer run.  delta is the per-motif failure probability of the
 * error bars (Corollary 5.3), 0.01 for 99% bars. */
typedef struct {
    uint64_t k_path;
    uint64_t k_cent;
    uint64_t seed;
    uint64_t first_id_path;
    uint64_t first_id_cent;
    double delta;
} pm_params;

/* Result of one count.  Arrays est/lo/hi/est_basic are indexed by motif
 * number 1..6 (index 0 unused).  est_basic[4..6] are Algorithm 2's own
 * estimates of the cycle-based motifs (the ones the paper discards). */
typedef struct {
    uint64_t tally_path[PM_NUM_TALLIES];
    uint64_t tally_cent[PM_NUM_TALLIES];
    uint64_t W;       /* sum over edges of (d_u - 1)(d_v - 1)      (Section 3) */
    uint64_t Lambda;  /* sum over edges of L_{u,v} L_{v,u}         (Section 4) */
    uint64_t N1;      /* sum over vertices of C(d_v, 3)           (Algorithm 2) */
    uint64_t k_path;
    uint64_t k_cent;
    double est[7];
    double lo[7];
    double hi[7];
    double est_basic[7];
} pm_result;

typedef struct {
    int64_t n;
    int64_t m;              /* undirected edges */
    int64_t dmax;
    int64_t isolated;       /* vertices of degree 0 */
    uint64_t W;
    uint64_t Lambda;
    uint64_t N1;
    uint64_t device_bytes;  /* resident device memory of the handle */
} pm_graph_info;

typedef struct pm_graph pm_graph;

/* ------------------------------------------------------------------------ */
/* One-shot                                                                  */
/* ------------------------------------------------------------------------ */

/* The whole method on one graph (end of Section 4): prepare the graph with
 * full validation, run both samplers with k samples each (seed, ids from 0),
 * and fill estimates with 99% Corollary 5.3 bars.  Default stream. */
pm_status pm_count_motifs(const pm_csr_view *csr, uint64_t k, uint64_t seed, pm_result *out);

/* ------------------------------------------------------------------------ */
/* Prepared graphs                                                           */
/* ------------------------------------------------------------------------ */

/* Prepare a graph on the current device: degrees, the degree-order relabel of
 * Section 4 (u before v iff d_u < d_v, or equal degrees and smaller input id;
 * rows re-sorted so that this order is integer order), the per-slot weights
 * tau = (d_u - 1)(d_v - 1) of Section 3 and lambda = L_{u,v} L_{v,u} of
 * Section 4 with their inclusive prefix sums, and N_1.
 * Limits: n < 2^31, 2m < 2^32.  Errors: PM_EINVAL (null / limits),
 * PM_EGRAPH (a failed check of flags), PM_EOVERFLOW, PM_ENOMEM, PM_EDEVICE.
 * The handle owns its device memory; release with pm_graph_destroy.  A handle
 * is immutable after creation: concurrent pm_count calls on it are safe. */
pm_status pm_graph_create(const pm_csr_view *csr, uint32_t flags, void *stream, pm_graph **out);

/* Sizes and totals of a prepared graph (the survey's pm_graph_info, named
 * _get here because the struct already takes that name): n, m, the largest
 * degree, isolated vertices, W (Section 3: 3-paths plus three times the
 * triangles, the total of tau over one orientation of each edge), Lambda
 * (Section 4: the total of lambda over one orientation), N_1 (Algorithm 2:
 * the sum over vertices of C(d_v, 3)) and the handle's resident device bytes.
 * Host call, no device work.  Errors: PM_EINVAL (null argument). */
pm_status pm_graph_info_get(const pm_graph *g, pm_graph_info *out);

/* Copy the prepared arrays to caller-owned host buffers (any pointer may be
 * NULL): off[n+1] and col[2m] of the graph relabelled in the degree order of
 * Section 4 (rows ascending), rank[n] (input id -> relabelled id), p_tau[2m]
 * (inclusive prefix of tau, Section 3 / Algorithm 1 step 1) and p_lam[2m]
 * (inclusive prefix of lambda, Section 4 / Algorithm 3 step 1), both global
 * over the slots.  Synchronises `stream` before returning.  Errors:
 * PM_EINVAL (null graph), PM_ENOMEM, PM_EDEVICE. */
pm_status pm_graph_export(const pm_graph *g, int64_t *off, int32_t *col, int32_t *rank, uint64_t *p_tau,
                          uint64_t *p_lam, void *stream);

/* Release a prepared graph (the arrays pm_graph_create built for Sections 3
 * and 4).  Waits for all work on the graph's device first (samplers still
 * running on any stream, pm_sample_async included), so the memory is never
 * handed out while a kernel reads it.  Errors: PM_EINVAL (null), PM_EDEVICE. */
pm_status pm_graph_destroy(pm_graph *g);

/* Run both samplers on a prepared graph and finalize on the host.  A sampler
 * whose total weight is 0 (W = 0 or Lambda = 0) draws nothing: its tallies,
 * estimates and bars are exactly 0.  k_path = k_cent = 0 is PM_EINVAL. */
pm_status pm_count(const pm_graph *g, const pm_params *p, pm_result *out, void *stream);

/* pm_count for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same samples, tallies and results as pm_count, with every device buffer
 * it needs in a fixed array inside the library instead of allocated: both
 * samplers' tallies and the buffers of one draw-order sort chunk of 2^22
 * sample ids, 68 MiB in all (pm_static_scratch_bytes).  Each device the
 * library runs on holds its own copy of the array until the process ends.
 * Budgets above one chunk are sorted and sampled chunk by chunk, so no k is
 * rejected for size.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); the array keeps the last call's contents and
 * the tallies are cleared at the start of each call.  Every call on one
 * device shares that device's array: calls that overlap on one device (from
 * several host threads or streams) race, so the caller serialises them.
 * Synchronises `stream`.  Errors as pm_count (PM_EINVAL, PM_EDEVICE). */
pm_status pm_count_noalloc(const pm_graph *g, const pm_params *p, pm_result *out, void *stream);

/* Bytes of the fixed per-device array pm_count_noalloc uses. */
uint64_t pm_static_scratch_bytes(void);

/* Alias-table edge draw: the variant of the weighted edge pick of
 * Algorithm 1 step 2 and Algorithm 3 step 2 by Walker's alias method (the
 * paper leaves the mechanism open).  pm_graph_build_alias adds one table per
 * sampler of nonzero total weight to a prepared graph (32 bytes per slot
 * each, counted in device_bytes, freed with the graph); calling it again is a
 * no-op.  The table is exact and fixed by the weights: N = 2m buckets of
 * capacity R (= 2W or 2 Lambda), slot s owning mass N w_s; light slots
 * (N w_s < R) in index order each keep their mass and fill their bucket from
 * the current heavy slot (index order), a heavy slot drawn below R filling
 * its own bucket from the next one.  Calls on one graph must not overlap
 * with each other or with samplers on it.  Errors: PM_EINVAL (null graph),
 * PM_ENOMEM, PM_EDEVICE. */
pm_status pm_graph_build_alias(pm_graph *g, void *stream);

/* pm_count through the alias tables.  Each sample draws, from its own
 * Philox stream (tag 2 for the 3-path sampler, 3 for the centered one; the
 * candidates of attempts 0, 1, ... in order), a bucket b in [0, 2m), a coin
 * x in [0, R) and then a position o in [0, w_s) inside the picked slot s, and
 * is decoded from (s, o) as in pm_count.  Tallies therefore differ from
 * pm_count's for the same seed, with the same distribution.  PM_EINVAL when
 * a sampler with nonzero weight has no table (pm_graph_build_alias first). */
pm_status pm_count_alias(const pm_graph *g, const pm_params *p, pm_result *out, void *stream);

/* Copy one sampler's alias table (centered = 0: tau, 1: lambda) to host
 * arrays K[2m] (kept mass of each bucket) and alias[2m].  PM_EINVAL when
 * that table was not built (or the sampler's total weight is 0). */
pm_status pm_graph_alias_export(const pm_graph *g, int32_t centered, uint64_t *K, int64_t *alias, void *stream);

/* Tallies only (no host finalize), written to the device buffer
 * tallies_dev[16] (path then centered, uint64) on the stream, without
 * synchronising.  The buffer is overwritten, not accumulated. */
pm_status pm_sample_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, void *stream);

/* ------------------------------------------------------------------------ */
/* Exact counts (ground truth)                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t C[7];      /* induced counts, index = motif number (1..6) */
    uint64_t N[7];      /* subgraph (not necessarily induced) counts of Eq. 1 */
    uint64_t triangles;
} pm_exact;

/* Exact counts of a prepared graph on the device, split as the paper's
 * enumeration code (Section 6): N_1 = sum C(d,3), N_2 = W - 3T,
 * N_3 = sum_v t_v (d_v - 2), N_5 = sum_e C(t_e, 2) from triangles per edge;
 * N_4 (4-cycles) and N_6 (4-cliques) by enumeration under the degree order;
 * then Eq. 1 solved for C.  Work grows like the wedge count (hours-free up
 * to ~1e8 edges of power-law graphs); device scratch of 8 n bytes per
 * counting block (256 blocks) besides 4 bytes per slot.  Synchronises the
 * stream.  Errors: PM_EINVAL, PM_EOVERFLOW (a count >= 2^64), PM_ENOMEM,
 * PM_EDEVICE. */
pm_status pm_exact_counts(const pm_graph *g, pm_exact *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Edge-list ingest                                                          */
/* ------------------------------------------------------------------------ */

/* A list of vertex pairs (src[e], dst[e]), e < num_edges, over vertices
 * 0..n-1.  Buffers on the device (on_device = 1) or the host (0, copied). */
typedef struct {
    int64_t n;
    int64_t num_edges;
    const int32_t *src;
    const int32_t *dst;
    int32_t on_device;
} pm_edge_view;

/* The undirected simple graph of an edge list, as CSR (the clean-up of the
 * paper's inputs, Section 6): every pair is an undirected edge, so both
 * directions become slots; self-loops are dropped; repeated pairs (in either
 * direction) are merged.  Rows come out strictly ascending.  off[n+1] and
 * col[capacity] are caller-owned device buffers; capacity = 2 * num_edges
 * always suffices; *slots_out = 2m.  Returns after the CSR is written (the
 * stream is synchronised).  Errors: PM_EINVAL (null, sizes, capacity too
 * small -- the message names the size needed), PM_EGRAPH (an endpoint
 * outside [0, n)), PM_ENOMEM, PM_EDEVICE. */
pm_status pm_csr_from_edges(const pm_edge_view *edges, int64_t *off, int32_t *col, int64_t capacity,
                            int64_t *slots_out, void *stream);

/* pm_csr_from_edges into library memory, then pm_graph_create on it (the
 * intermediate CSR is freed).  The end-to-end path from a raw edge list. */
pm_status pm_graph_from_edges(const pm_edge_view *edges, uint32_t flags, void *stream, pm_graph **out);

/* ------------------------------------------------------------------------ */
/* Batched sampling: many prepared graphs in one launch                      */
/* ------------------------------------------------------------------------ */

/* Launch shape of a batch: samples per work tile and resident blocks per
 * compute unit.  samples_per_tile = 0 asks the autotuner, which times tile
 * sizes {1024, 4096, 16384} x blocks {2, 4, 8} on the batch and keeps the
 * fastest (cached per graph count and total-sample magnitude). */
typedef struct {
    int32_t samples_per_tile;
    int32_t blocks_per_cu;
} pm_tune;

typedef struct pm_batch pm_batch;

/* A batch over count prepared graphs (all on the current device), graph i
 * sampled with params[i].  Every graph's result is bit-for-bit the result of
 * pm_count(graphs[i], &params[i]): samples depend only on (seed, sampler,
 * id).  The work is a table of tiles (graph, sampler, first id, count, seed)
 * consumed by one persistent kernel; the whole run (table upload, tally
 * reset, kernel, tally download) is captured once as a HIP graph on an
 * internal stream and replayed by pm_batch_run.  The batch keeps pointers to
 * the graphs: destroy the batch before them.  Errors: PM_EINVAL (null,
 * count <= 0, a graph on another device, k_path = k_cent = 0, delta outside
 * (0,1), bad tune), PM_ENOMEM, PM_EDEVICE. */
pm_status pm_batch_create(const pm_graph *const *graphs, const pm_params *params, int32_t count, const pm_tune *tune,
                          void *stream, pm_batch **out);

/* New parameters for the same graphs (seeds, id ranges, budgets); no
 * recapture.  PM_EINVAL when the new budgets need more tiles than the batch
 * was created with (the capacity is that of the creation budgets cut into
 * tiles of min(1024, the requested tile size) samples). */
pm_status pm_batch_set_params(pm_batch *b, const pm_params *params);

/* Replay the batch after the work already on `stream`; out[count] receives
 * each graph's result.  Returns when the results are on the host. */
pm_status pm_batch_run(pm_batch *b, pm_result *out, void *stream);

pm_status pm_batch_get_tune(const pm_batch *b, pm_tune *out);
pm_status pm_batch_destroy(pm_batch *b);

/* One-shot: pm_batch_create, pm_batch_run, pm_batch_destroy. */
pm_status pm_count_batch(const pm_graph *const *graphs, const pm_params *params, pm_result *out, int32_t count,
                         const pm_tune *tune, void *stream);

/* ------------------------------------------------------------------------ */
/* Served mode: continuous batching of motif-count requests                  */
/* ------------------------------------------------------------------------ */

/* A server owns registered graphs, prepares them on the device when a
 * request needs them (and keeps them resident within an HBM budget), and
 * runs requests in steps: each step is one persistent launch over work tiles
 * of every active request, so requests that arrive while others run are
 * admitted between steps and share the device with them.  A request either
 * gives its sample budgets or asks for a relative error: then its first
 * k_pilot ids per sampler are a pilot from which k is sized with
 * Corollary 5.3 (pm_samples_for_request) and the ids [k_pilot, k) follow.
 * A finished request's result is bit-for-bit pm_count with its final
 * (k_path, k_cent, seed, first ids 0, delta): tallies are sums over ids, so
 * how the ids are cut into steps does not matter. */
typedef struct pm_server pm_server;

typedef struct {
    uint64_t hbm_budget;     /* bytes for resident prepared graphs (0: 3/4 of free device memory) */
    int32_t max_active;      /* requests on the device at once (0: 256) */
    int32_t max_graphs;      /* registered graphs (0: 1024) */
    uint64_t step_samples;   /* samples per step shared by the active requests (0: 2^25) */
    uint64_t k_pilot;        /* pilot ids per sampler (0: 65536) */
    uint64_t k_max;          /* cap on a sized budget, per sampler (0: 2e9) */
    int32_t samples_per_tile;  /* work tile (0: 4096) */
    int32_t blocks_per_cu;     /* resident blocks per compute unit (0: 4) */
} pm_server_cfg;

typedef struct {
    uint32_t graph;       /* id from pm_server_add_graph */
    uint32_t motif_mask;  /* bit i (i = 1..6): size k for motif i; 0 means all six */
    double rel_err;       /* requested relative error, (0,1) (ignored with fixed budgets) */
    double delta;         /* failure probability per motif, (0,1) */
    uint64_t seed;        /* Philox key */
    uint64_t k_path;      /* fixed budgets: if either is non-zero both are used as */
    uint64_t k_cent;      /* given and no pilot is run */
} pm_request;

typedef struct {
    double queued_ms;      /* submit to admission */
    double latency_ms;     /* submit to result */
    uint64_t k_path, k_cent; /* final budgets */
    uint32_t steps;        /* device steps that carried its work */
    uint32_t capped_mask;  /* bit i: motif i needed more than k_max (its bar is what k_max gives) */
    uint32_t unseen_mask;  /* bit i: motif i had no pilot hit (sized from the pilot's upper bound) */
    int32_t prepared;      /* 1: its admission prepared (or re-prepared) the graph */
} pm_req_stats;

typedef struct {
    uint64_t steps, samples, requests_done;
    uint64_t resident_bytes, resident_graphs, preparations, evictions;
    double busy_ms;        /* sum of step durations (device events) */
} pm_server_stats;

/* Create a server on the current device; its worker thread starts at once.
 * cfg may be NULL (all defaults).  Errors: PM_EINVAL, PM_ENOMEM, PM_EDEVICE. */
pm_status pm_server_create(const pm_server_cfg *cfg, pm_server **out);

/* Register a graph.  The CSR buffers (host or device) are read when the graph
 * is prepared, which may happen again after an eviction: they must stay
 * valid and unchanged until pm_server_destroy.  flags as for
 * pm_graph_create.  Errors: PM_EINVAL (null, too many graphs). */
pm_status pm_server_add_graph(pm_server *srv, const pm_csr_view *csr, uint32_t flags, uint32_t *graph_id);

/* Prepare a registered graph now (blocking).  PM_EBUSY when it cannot fit
 * beside the graphs pinned by active requests, PM_ENOMEM when it exceeds the
 * budget alone, or the pm_graph_create error for an invalid graph. */
pm_status pm_server_preload(pm_server *srv, uint32_t graph_id);

/* Queue a request (non-blocking); admission is first come, first served,
 * when a slot is free and the graph is resident or fits the budget after
 * evicting idle graphs (least recently used first).  Errors: PM_EINVAL
 * (unknown graph, rel_err or delta outside (0,1) when sizing), PM_ECANCELED
 * (server shutting down). */
pm_status pm_server_submit(pm_server *srv, const pm_request *req, uint64_t *ticket);

/* Wait for a request and release its ticket.  timeout_ms < 0 waits for
 * ever; on timeout PM_EBUSY is returned and the ticket stays valid.  The
 * request's own status is returned otherwise (PM_OK, PM_ECANCELED, the error
 * of preparing its graph, PM_ENOMEM if its graph exceeds the budget alone).
 * out and st may be NULL. */
pm_status pm_server_wait(pm_server *srv, uint64_t ticket, int64_t timeout_ms, pm_result *out, pm_req_stats *st);

/* Cancel a queued or running request (its wait returns PM_ECANCELED unless
 * it already finished). */
pm_status pm_server_cancel(pm_server *srv, uint64_t ticket);

pm_status pm_server_get_stats(pm_server *srv, pm_server_stats *out);

/* Cancel what is left, stop the worker, free every prepared graph.  No
 * other call on this server may be in progress or follow. */
pm_status pm_server_destroy(pm_server *srv);

/* The sizing rule of the served mode.  From pilot tallies over k0 ids per
 * sampler: alpha_i = t_i / k0 for the motifs of mask (2, 3 from the 3-path
 * sampler; 4, 5, 6 from the centered one); a motif with no hit uses the
 * upper end p_u of its Definition 5.2 interval instead (bit i of *unseen);
 * k_i = pm_samples_for_error(rel_err, delta, alpha_i).  Motif 1 is the
 * difference N_1 - C_3 - 2 C_5 - 4 C_6 of Algorithm 2: its error budget
 * rel_err * est_1 (pilot estimates) is split evenly over the h terms with a
 * hit, term j sized at relative error rel_err * est_1 / (h c_j est_j),
 * c = (1, 2, 4), when that is below 1; est_1 <= 0 sets bit 1 of *capped.
 * alpha = 1 uses D(1, 1 - e) = ln(1 / (1 - e)).  A sampler's k is the
 * largest k_i of its motifs and at least k0; a k_i above k_max becomes k_max
 * (bit i of *capped).  A sampler of zero total weight gets k0.  Errors:
 * PM_EINVAL (null, k0 = 0, k_max < k0, rel_err or delta outside (0,1)). */
pm_status pm_samples_for_request(const uint64_t tally_path[PM_NUM_TALLIES], const uint64_t tally_cent[PM_NUM_TALLIES],
                                 uint64_t k0, uint64_t W, uint64_t Lambda, uint64_t N1, uint32_t motif_mask,
                                 double rel_err, double delta, uint64_t k_max, uint64_t *k_path, uint64_t *k_cent,
                                 uint32_t *capped, uint32_t *unseen);

/* ------------------------------------------------------------------------ */
/* Host-side estimates and error bars                                        */
/* ------------------------------------------------------------------------ */

/* Estimates of Algorithms 2 and 4 and the bars of Corollary 5.3 from tallies
 * (fills every field of out).  W, Lambda, N1 as in pm_result. */
pm_status pm_finalize(const uint64_t tally_path[PM_NUM_TALLIES], const uint64_t tally_cent[PM_NUM_TALLIES],
                      uint64_t W, uint64_t Lambda, uint64_t N1, uint64_t k_path, uint64_t k_cent, double delta,
                      pm_result *out);

/* (p_l, p_u) of Definition 5.2: the roots of k D(count/k, p) = ln(1/delta). */
pm_status pm_chernoff_interval(uint64_t count, uint64_t k, double delta, double *p_lo, double *p_hi);

/* Smallest k whose Corollary 5.3 bar around a proportion alpha stays within
 * relative error rel_err at failure probability delta:
 * k = ceil(ln(1/delta) / min(D(alpha, alpha(1+e)), D(alpha, alpha(1-e)))). */
pm_status pm_samples_for_error(double rel_err, double delta, double alpha, uint64_t *k_out);

/* Launch shape of the two sampling kernels for this process: samples each
 * lane advances together (1, 2 or 4; more loads in flight per lane, more
 * registers; id-order launches only) and resident blocks per compute unit
 * (1..64; also the grid of the draw-ordered launches).  Tallies do not depend
 * on the shape.  Default 1 and 4 (the fastest measured on MI355X). */
pm_status pm_set_sampler_shape(int32_t samples_per_lane, int32_t blocks_per_cu);

/* Draw-ordered sampling in pm_count, pm_sample_async and pm_count_alias
 * (this process; on by default).  When a sampler draws at least min_samples
 * samples (0: the default 2^21, about where the sort starts to pay on
 * MI355X), their ids are first sorted, in chunks of 2^24, by the top 24 bits
 * of each sample's first draw (r of Algorithm 1 step 2 / Algorithm 3 step 2,
 * or the alias bucket), so that neighbouring lanes read neighbouring parts of
 * the graph; each sample then runs as usual.  Tallies are sums over ids and
 * do not change: enabled = 0 gives the same results in id order. */
pm_status pm_set_draw_order(int32_t enabled, uint64_t min_samples);

/* The order in which a draw-ordered launch runs one sort chunk of a sampler
 * (samples first_id .. first_id + k - 1, 1 <= k <= 2^24): ids_out[j] =
 * id - first_id of the j-th sample run.  The ids are in nondecreasing order
 * of the draw key of pm_set_draw_order (the top 24 bits of the sample's r of
 * Algorithm 1 step 2 for centered = 0, Algorithm 3 step 2 for centered = 1;
 * all of r when the sampler's total weight is below 2^24); the order among
 * equal keys is unspecified.  ids_out is a device array of k entries, written
 * asynchronously on `stream`.  Errors: PM_EINVAL (null arguments, k out of
 * range, a sampler whose total weight is below 2, another device's graph),
 * PM_ENOMEM, PM_EDEVICE. */
pm_status pm_draw_order(const pm_graph *g, int32_t centered, uint64_t seed, uint64_t first_id, uint64_t k,
                        uint32_t *ids_out, void *stream);

/* How pm_count and pm_sample_async run the adjacency tests of Algorithms 2
 * and 4 ("determine the subgraph induced by" the sampled path) in this
 * process.  The paper keeps adjacency in hash tables (Theorem 3.5); here:
 * PM_SEARCH_HASH (2, the default) probes a per-row hash of the row's columns
 * (open addressing at load 1/2, built with the graph): one aligned 16-byte
 * read nearly always decides.  PM_SEARCH_LANE (0) searches the sorted row in
 * each sample's own lane through the row search index (one 128-byte line per
 * level, read as eight 16-byte loads per lane).  PM_SEARCH_WAVE (1) lets the
 * 64 lanes of a wave read each query's index line together (two queries per
 * coalesced load, a ballot counts the entries at most the key); on MI355X it
 * measured about three times slower than PM_SEARCH_LANE (its rounds spend
 * their time in cross-lane instructions).  All give the same answers, so
 * tallies do not change.  The batched, served and alias paths always probe
 * the row hash.  Errors: PM_EINVAL for another mode. */
#define PM_SEARCH_LANE 0
#define PM_SEARCH_WAVE 1
#define PM_SEARCH_HASH 2
pm_status pm_set_search_mode(int32_t mode);

/* Device memory: the library keeps freed blocks for reuse (each tagged with
 * an event on the stream that released it).  This returns every cached block
 * of the current device to the runtime (after those events complete).  Blocks
 * are freed on the device that allocated them. */
pm_status pm_release_cached_memory(void);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 block function evaluated on the device for count inputs of
 * six words (c0 c1 c2 c3 k0 k1) each, host arrays in and out (4 words per
 * input). */
pm_status pm_philox_device(const uint32_t *in, uint32_t *out, int64_t count);

/* Streaming copy of `bytes` bytes between two device buffers on `stream`
 * (16-byte vector loads and stores, asynchronous): the reference kernel of
 * known traffic for calibrating hardware counters and for the measured
 * streaming ceiling.  Pointers aligned to 16 bytes, bytes a multiple of 16,
 * else PM_EINVAL. */
pm_status pm_device_copy(void *dst, const void *src, uint64_t bytes, void *stream);

/* count independent 4-byte loads at pseudo-random positions (a splitmix64
 * stream from seed) of a device table of `bytes` bytes, asynchronous on
 * `stream`: the measured ceiling for line-granular random access, against
 * which the samplers' line traffic is read.  Table 4-byte aligned, at least
 * 4 bytes, count >= 0, else PM_EINVAL. */
pm_status pm_device_gather(const void *table, uint64_t bytes, int64_t count, uint64_t seed, void *stream);

/* The adjacency test of the samplers on its own (Algorithms 2 and 4
 * "determine the subgraph induced by" the path): out[i] = 1 if relabelled
 * vertices a[i] and b[i] are adjacent in the prepared graph, else 0, found
 * with search mode `mode` (PM_SEARCH_LANE, PM_SEARCH_WAVE or PM_SEARCH_HASH;
 * each searches the row of the smaller id, as the samplers do).  a, b and
 * out are device arrays of `count` entries (ids in [0, n), a[i] != b[i];
 * relabelled ids are positions in the degree order, see pm_graph_export's
 * rank); asynchronous on `stream`.  Errors: PM_EINVAL (null arguments,
 * count < 0, unknown mode), PM_EDEVICE.  Ids are not range-checked on the
 * device: out-of-range ids are undefined behaviour. */
pm_status pm_adjacent(const pm_graph *g, const int32_t *a, const int32_t *b, int64_t count, uint8_t *out,
                      int32_t mode, void *stream);

/* Per-kernel timing with HIP events recorded on each launch's stream.
 * pm_profile_enable clears the totals and switches recording on (1) or off
 * (0); pm_profile_read waits for the recorded events and returns one entry
 * per kernel name (count = number of names, entries beyond capacity are
 * dropped).  Timing adds two event records per launch. */
typedef struct {
    char name[48];
    uint64_t launches;
    double total_ms;
} pm_profile_entry;

pm_status pm_profile_enable(int32_t on);
pm_status pm_profile_read(pm_profile_entry *out, int32_t capacity, int32_t *count);

/* Restrict the recording to the named scopes: `names` is a comma-separated
 * list of kernel names as pm_profile_read reports them (e.g.
 * "reverse_sort.scatter,sample_path"); null or "" records every scope again.
 * The selection stays until the next call and does not clear the totals.
 * Each recorded scope adds two event records between kernels on its stream,
 * so timing a few scopes perturbs the timed work less than timing all.
 * Always PM_OK. */
pm_status pm_profile_select(const char *names);

const char *pm_status_string(pm_status s);
const char *pm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PATHSAMP_H */
