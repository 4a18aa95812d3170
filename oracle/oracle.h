/*
 * Plain single-threaded CPU oracle for 3-path sampling (Jha, Seshadhri, Pinar,
 * "Path Sampling: A Fast and Provable Method for Estimating 4-Vertex Subgraph
 * Counts").
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the HIP library.
 *
 * Every quantity is integer and exact.  Vertex ids are int32, slot positions
 * and offsets int64, weights / prefixes / tallies uint64.
 */
#ifndef PATHSAMP_ORACLE_H
#define PATHSAMP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_EGRAPH (-2)
#define OR_EOVERFLOW (-3)
#define OR_ENOMEM (-4)

/* Sample outcome classes.  Index i in 2..6 is motif i of the paper's Figure 1
 * numbering (1 3-star, 2 3-path, 3 tailed-triangle, 4 4-cycle,
 * 5 chordal-4-cycle, 6 4-clique).  Index 0 is the triangle outcome (u'=v');
 * index 1 is the centered sampler's "not centered" rejection. */
#define OR_TRI 0
#define OR_OPEN 1

/* Canonical prepared graph: the input relabelled into the paper's degree
 * order (Section 4), with both weight prefixes. */
typedef struct {
    int64_t n;          /* vertices */
    int64_t slots;      /* directed adjacency slots = 2m */
    int64_t *off;       /* [n+1] row offsets of the relabelled graph */
    int32_t *col;       /* [slots] neighbours, each row ascending */
    int32_t *rank;      /* [n] input id -> canonical id */
    uint64_t *p_tau;    /* [slots] inclusive prefix of tau over slots */
    uint64_t *p_lam;    /* [slots] inclusive prefix of lambda over slots */
    uint64_t R_tau;     /* = 2W  (each undirected edge has two slots) */
    uint64_t R_lam;     /* = 2 Lambda */
    uint64_t N1;        /* sum over v of C(d_v, 3) */
} or_graph;

/* Input checks: offsets start at 0 and never decrease, every column is a
 * vertex id, rows strictly increase (no duplicate edge), no self-loop, and
 * the adjacency is symmetric (undirected simple graph, Section 2). */
int or_validate(int64_t n, const int64_t *off, const int32_t *col);

/* Validate, relabel, compute tau/lambda prefixes and N1.  On success the
 * graph owns its arrays; release with or_graph_free. */
int or_graph_build(int64_t n, const int64_t *off, const int32_t *col, or_graph *g);
void or_graph_free(or_graph *g);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Lemire's bounded draw on a word of `bits` bits (1..64): returns 1 and sets
 * *r in [0,R) when x is accepted, 0 when x must be redrawn.  Requires
 * 1 <= R <= 2^bits. */
int or_lemire(uint64_t x, uint64_t R, int bits, uint64_t *r);

/* Exact uniform integer in [0,R) for sample `id` of sampler `tag`. */
uint64_t or_draw(uint64_t seed, uint32_t tag, uint64_t id, uint64_t R);

/* out[i] = or_draw(seed, tag, first + i, R) for i < k. */
void or_draws(uint64_t seed, uint32_t tag, uint64_t first, uint64_t k, uint64_t R, uint64_t *out);

/* Map r in [0,R_tau) to the 3-path (u', u, v, v') of Algorithm 1;
 * q[0]=u', q[1]=u, q[2]=v, q[3]=v'. */
void or_decode_path(const or_graph *g, uint64_t r, int32_t q[4]);
/* Map r in [0,R_lam) to the output of Algorithm 3 (same layout). */
void or_decode_centered(const or_graph *g, uint64_t r, int32_t q[4]);

/* Outcome class of a decoded sample (index into a tally[8]). */
int or_classify_path(const or_graph *g, const int32_t q[4]);
int or_classify_centered(const or_graph *g, const int32_t q[4]);

/* k samples with ids first..first+k-1; tally[8] is overwritten.  A sampler
 * whose total weight is 0 leaves its tally at zero. */
void or_sample_path(const or_graph *g, uint64_t seed, uint64_t first, uint64_t k, uint64_t tally[8]);
void or_sample_centered(const or_graph *g, uint64_t seed, uint64_t first, uint64_t k, uint64_t tally[8]);

/* Every r in [0,R) once: the exact distribution of one sample times R. */
void or_enumerate_path(const or_graph *g, uint64_t tally[8]);
void or_enumerate_centered(const or_graph *g, uint64_t tally[8]);

/* Alias-table edge draw (alias.c): the variant of the weighted edge pick.
 * or_alias_build fills K[N] and alias[N] for weights w[N] (total R in
 * (0, 2^64)); or_draw_alias returns r = P[s-1] + o for sample `id` from the
 * table (b, x and o drawn in that order from the sample's Philox stream);
 * the alias samplers decode r exactly as the main samplers do, with tags 2
 * (3-path) and 3 (centered). */
int or_alias_build(const uint64_t *w, int64_t N, uint64_t *K, int64_t *alias);
uint64_t or_draw_alias(const uint64_t *P, const uint64_t *K, const int64_t *alias, int64_t N, uint64_t R,
                       uint64_t seed, uint32_t tag, uint64_t id);
void or_sample_path_alias(const or_graph *g, const uint64_t *K, const int64_t *alias, uint64_t seed, uint64_t first,
                          uint64_t k, uint64_t tally[8]);
void or_sample_centered_alias(const or_graph *g, const uint64_t *K, const int64_t *alias, uint64_t seed,
                              uint64_t first, uint64_t k, uint64_t tally[8]);

/* Exact induced counts C[1..6] (C[0] unused) and triangle count.
 * Brute force over every 4-subset (n <= 512). */
int or_exact_brute(int64_t n, const int64_t *off, const int32_t *col, uint64_t C[7], uint64_t *T);
/* Exact counts from subgraph (non-induced) counts N_1..N_6 and Eq. 1. */
int or_exact_formula(int64_t n, const int64_t *off, const int32_t *col, uint64_t C[7], uint64_t *T);

#ifdef __cplusplus
}
#endif
#endif
