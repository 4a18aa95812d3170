/*
 * Plain single-threaded CPU oracle for 3-path sampling (Jha, Seshadhri, Pinar,
 * "Path Sampling: A Fast and Provable Method for Estimating 4-Vertex Subgraph
 * Counts").
 *
 * TEST INFRASTRUCTURE ONLY: the checker the HIP library is compared against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code with the HIP library.
 *
 * It favours the obvious over the fast: binary searches are written out,
 * sorting uses qsort, every accumulation is 128-bit with explicit overflow
 * checks.  The steps follow the paper's order:
 *   Section 2  : simple undirected input, motif numbering, Eq. 1
 *   Section 3  : tau_e, W, Algorithm 1 (sample) and Algorithm 2 (3-path-sampler)
 *   Section 4  : the degree order, L_{u,v}, lambda_e, Lambda, Algorithm 3
 *                (sample-centered) and Algorithm 4 (centered-sampler)
 * Estimates and error bars (Algorithms 2/4, Section 5) are computed from the
 * tallies by the Python half of the oracle.
 *
 * Readings fixed here where the paper is silent (each listed in the design
 * notes of the repository):
 *  - "pick e with probability p_e": inverse CDF over the directed slots of
 *    the relabelled CSR (both orientations of every edge, which leaves every
 *    probability of Claims 3.1 and 4.3 unchanged).
 *  - One uniform r in [0, R) per sample decodes (slot, u', v') in mixed
 *    radix, an exact bijection onto the sample space of Algorithm 1/3.
 *  - Random numbers: Philox4x32-10 keyed by the seed, counter (id, tag,
 *    attempt); exact bounded integers by Lemire's multiply-and-reject.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define U64_LIMIT (((u128)1) << 64)

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

static int64_t degree(const int64_t *off, int64_t v) { return off[v + 1] - off[v]; }

/* first index s in [lo, hi) with a[s] > x, or hi */
static int64_t upper_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t x)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] > x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

/* first index s in [0, len) with p[s] > r, or len */
static int64_t upper_bound_u64(const uint64_t *p, int64_t len, uint64_t r)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (p[mid] > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

/* is b a neighbour of a?  (rows ascending) */
static int adjacent(const int64_t *off, const int32_t *col, int32_t a, int32_t b)
{
    int64_t lo = off[a], hi = off[a + 1];
    int64_t s = upper_bound_i32(col, lo, hi, b);
    return s > lo && col[s - 1] == b;
}

/* L_{a,b} of Section 4: the number of neighbours of a that are greater than
 * b.  In the relabelled graph "greater in the degree order" is integer >. */
static int64_t count_greater(const or_graph *g, int32_t a, int32_t b)
{
    int64_t lo = g->off[a], hi = g->off[a + 1];
    return hi - upper_bound_i32(g->col, lo, hi, b);
}

/* row containing slot s: the u with off[u] <= s < off[u+1] */
static int32_t row_of_slot(const or_graph *g, int64_t s)
{
    int64_t lo = 0, hi = g->n + 1; /* first x with off[x] > s */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->off[mid] > s)
            hi = mid;
        else
            lo = mid + 1;
    }
    return (int32_t)(lo - 1);
}

/* Motif of a connected 4-vertex graph from its sorted degree sequence
 * (Figure 1 numbering); 0 for a disconnected 4-set.  A connected graph on
 * four vertices is determined up to isomorphism by its degree sequence. */
static int motif_of_degrees(int d[4])
{
    for (int i = 0; i < 4; i++) /* insertion sort, ascending */
        for (int j = i; j > 0 && d[j - 1] > d[j]; j--) {
            int t = d[j];
            d[j] = d[j - 1];
            d[j - 1] = t;
        }
    int key = d[0] * 1000 + d[1] * 100 + d[2] * 10 + d[3];
    switch (key) {
    case 1113: return 1; /* 3-star          */
    case 1122: return 2; /* 3-path          */
    case 1223: return 3; /* tailed-triangle */
    case 2222: return 4; /* 4-cycle         */
    case 2233: return 5; /* chordal-4-cycle */
    case 3333: return 6; /* 4-clique        */
    default: return 0;
    }
}

/* induced motif on four distinct vertices, edges looked up in the graph */
static int induced_motif(const int64_t *off, const int32_t *col, const int32_t q[4])
{
    int d[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; i++)
        for (int j = i + 1; j < 4; j++)
            if (adjacent(off, col, q[i], q[j])) {
                d[i]++;
                d[j]++;
            }
    return motif_of_degrees(d);
}

/* ------------------------------------------------------------------------ */
/* input validation (Section 2: undirected simple graph)                    */
/* ------------------------------------------------------------------------ */

int or_validate(int64_t n, const int64_t *off, const int32_t *col)
{
    if (n < 0 || n > INT32_MAX || off == NULL)
        return OR_EINVAL;
    if (off[0] != 0)
        return OR_EGRAPH;
    for (int64_t v = 0; v < n; v++)
        if (off[v + 1] < off[v])
            return OR_EGRAPH;
    if (off[n] > 0 && col == NULL)
        return OR_EINVAL;
    for (int64_t v = 0; v < n; v++) {
        for (int64_t s = off[v]; s < off[v + 1]; s++) {
            int32_t c = col[s];
            if (c < 0 || c >= n || c == v)
                return OR_EGRAPH;
            if (s > off[v] && col[s - 1] >= c)
                return OR_EGRAPH;
        }
    }
    for (int64_t v = 0; v < n; v++)
        for (int64_t s = off[v]; s < off[v + 1]; s++)
            if (!adjacent(off, col, col[s], (int32_t)v))
                return OR_EGRAPH;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* canonical relabel into the degree order of Section 4                     */
/* ------------------------------------------------------------------------ */

/* per thread: tests prepare several oracle graphs on host threads at once */
static _Thread_local const int64_t *g_sort_off;

static int cmp_degree_then_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    int64_t da = degree(g_sort_off, a), db = degree(g_sort_off, b);
    if (da != db)
        return da < db ? -1 : 1;
    return (a > b) - (a < b);
}

static int cmp_i32(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

void or_graph_free(or_graph *g)
{
    if (!g)
        return;
    free(g->off);
    free(g->col);
    free(g->rank);
    free(g->p_tau);
    free(g->p_lam);
    memset(g, 0, sizeof(*g));
}

int or_graph_build(int64_t n, const int64_t *off_in, const int32_t *col_in, or_graph *g)
{
    if (g == NULL)
        return OR_EINVAL;
    memset(g, 0, sizeof(*g));
    int st = or_validate(n, off_in, col_in);
    if (st != OR_OK)
        return st;
    int64_t slots = off_in[n];
    g->n = n;
    g->slots = slots;
    g->off = malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->col = malloc(sizeof(int32_t) * (size_t)(slots > 0 ? slots : 1));
    g->rank = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->p_tau = malloc(sizeof(uint64_t) * (size_t)(slots > 0 ? slots : 1));
    g->p_lam = malloc(sizeof(uint64_t) * (size_t)(slots > 0 ? slots : 1));
    int32_t *order = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!g->off || !g->col || !g->rank || !g->p_tau || !g->p_lam || !order) {
        free(order);
        or_graph_free(g);
        return OR_ENOMEM;
    }

    /* u < v in the new ids iff d_u < d_v, or equal degrees and smaller input
     * id: the order of Section 4. */
    for (int64_t v = 0; v < n; v++)
        order[v] = (int32_t)v;
    g_sort_off = off_in;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_degree_then_id);
    for (int64_t i = 0; i < n; i++)
        g->rank[order[i]] = (int32_t)i;

    g->off[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t old = order[i];
        int64_t d = degree(off_in, old);
        int64_t base = g->off[i];
        for (int64_t t = 0; t < d; t++)
            g->col[base + t] = g->rank[col_in[off_in[old] + t]];
        qsort(g->col + base, (size_t)d, sizeof(int32_t), cmp_i32);
        g->off[i + 1] = base + d;
    }
    free(order);

    /* Section 3: tau_e = (d_u - 1)(d_v - 1); prefix over slots, total 2W. */
    u128 acc = 0;
    for (int64_t u = 0; u < n; u++) {
        int64_t du = degree(g->off, u);
        for (int64_t s = g->off[u]; s < g->off[u + 1]; s++) {
            int64_t dv = degree(g->off, g->col[s]);
            acc += (u128)(uint64_t)(du - 1) * (uint64_t)(dv - 1);
            if (acc >= U64_LIMIT) {
                or_graph_free(g);
                return OR_EOVERFLOW;
            }
            g->p_tau[s] = (uint64_t)acc;
        }
    }
    g->R_tau = (uint64_t)acc;

    /* Section 4: lambda_e = L_{u,v} L_{v,u}; prefix, total 2 Lambda. */
    acc = 0;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t s = g->off[u]; s < g->off[u + 1]; s++) {
            int32_t v = g->col[s];
            int64_t luv = count_greater(g, (int32_t)u, v);
            int64_t lvu = count_greater(g, v, (int32_t)u);
            acc += (u128)(uint64_t)luv * (uint64_t)lvu;
            if (acc >= U64_LIMIT) {
                or_graph_free(g);
                return OR_EOVERFLOW;
            }
            g->p_lam[s] = (uint64_t)acc;
        }
    }
    g->R_lam = (uint64_t)acc;

    /* Algorithm 2: N_1 = sum over v of C(d_v, 3), the 3-star subgraphs. */
    acc = 0;
    for (int64_t v = 0; v < n; v++) {
        u128 d = (u128)degree(g->off, v);
        if (d >= 3)
            acc += d * (d - 1) * (d - 2) / 6;
        if (acc >= U64_LIMIT) {
            or_graph_free(g);
            return OR_EOVERFLOW;
        }
    }
    g->N1 = (uint64_t)acc;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* randomness                                                               */
/* ------------------------------------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
 * multiplies words 0 and 2 by two fixed 32-bit constants, mixes the high
 * halves with the other two words and the round key, and the key is bumped
 * by two Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Lemire (ACM TOMACS 2019): r = floor(x R / 2^bits); x is rejected when the
 * low part of x R falls below (2^bits - R) mod R, which makes every r in
 * [0, R) have exactly floor(2^bits / R) accepted preimages. */
int or_lemire(uint64_t x, uint64_t R, int bits, uint64_t *r)
{
    u128 two_b = ((u128)1) << bits;
    u128 p = (u128)x * R;
    u128 low = p & (two_b - 1);
    if (low < R) {
        u128 t = (two_b - R) % R;
        if (low < t)
            return 0;
    }
    *r = (uint64_t)(p >> bits);
    return 1;
}

uint64_t or_draw(uint64_t seed, uint32_t tag, uint64_t id, uint64_t R)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t attempt = 0;; attempt++) {
        uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), tag, attempt};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        uint64_t x0 = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        uint64_t x1 = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
        uint64_t r;
        if (or_lemire(x0, R, 64, &r))
            return r;
        if (or_lemire(x1, R, 64, &r))
            return r;
    }
}

/* r of samples first .. first + k - 1 of one sampler, each as or_draw */
void or_draws(uint64_t seed, uint32_t tag, uint64_t first, uint64_t k, uint64_t R, uint64_t *out)
{
    for (uint64_t i = 0; i < k; i++)
        out[i] = or_draw(seed, tag, first + i, R);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (sample) and Algorithm 2's classification                    */
/* ------------------------------------------------------------------------ */

void or_decode_path(const or_graph *g, uint64_t r, int32_t q[4])
{
    /* pick the edge (slot) with probability tau / 2W */
    int64_t s = upper_bound_u64(g->p_tau, g->slots, r);
    int32_t u = row_of_slot(g, s);
    int32_t v = g->col[s];
    uint64_t o = r - (s > 0 ? g->p_tau[s - 1] : 0);
    int64_t du = degree(g->off, u), dv = degree(g->off, v);
    /* o in [0, (du-1)(dv-1)): digit a picks u', digit b picks v' */
    uint64_t a = o / (uint64_t)(dv - 1);
    uint64_t b = o % (uint64_t)(dv - 1);
    /* a-th element of N(u) \ {v}: positions 0..du-2, with v's own position
     * (if among them) standing for the last element of the row */
    int32_t up = g->col[g->off[u] + (int64_t)a];
    if (up == v)
        up = g->col[g->off[u] + du - 1];
    int32_t vp = g->col[g->off[v] + (int64_t)b];
    if (vp == u)
        vp = g->col[g->off[v] + dv - 1];
    q[0] = up;
    q[1] = u;
    q[2] = v;
    q[3] = vp;
}

int or_classify_path(const or_graph *g, const int32_t q[4])
{
    if (q[0] == q[3])
        return OR_TRI; /* u' = v': the output is a triangle */
    int m = induced_motif(g->off, g->col, q);
    return m; /* 2..6: a 3-path lies in every motif but the 3-star */
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3 (sample-centered) and Algorithm 4's classification           */
/* ------------------------------------------------------------------------ */

void or_decode_centered(const or_graph *g, uint64_t r, int32_t q[4])
{
    int64_t s = upper_bound_u64(g->p_lam, g->slots, r);
    int32_t u = row_of_slot(g, s);
    int32_t v = g->col[s];
    uint64_t o = r - (s > 0 ? g->p_lam[s - 1] : 0);
    int64_t du = degree(g->off, u), dv = degree(g->off, v);
    int64_t luv = count_greater(g, u, v);
    int64_t lvu = count_greater(g, v, u);
    /* o in [0, luv * lvu) */
    uint64_t a = o / (uint64_t)lvu;
    uint64_t b = o % (uint64_t)lvu;
    /* the neighbours of u greater than v are the last luv entries of the
     * ascending row, those of v greater than u the last lvu entries */
    int32_t up = g->col[g->off[u] + (du - luv) + (int64_t)a];
    int32_t vp = g->col[g->off[v] + (dv - lvu) + (int64_t)b];
    q[0] = up;
    q[1] = u;
    q[2] = v;
    q[3] = vp;
}

int or_classify_centered(const or_graph *g, const int32_t q[4])
{
    if (q[0] == q[3])
        return OR_TRI;
    /* Definition 4.1: with v < u' and u < v' by construction, the output
     * is centered iff (u', v') is an edge (it closes a 4-cycle) */
    if (!adjacent(g->off, g->col, q[0], q[3]))
        return OR_OPEN;
    return induced_motif(g->off, g->col, q); /* 4, 5 or 6 */
}

/* ------------------------------------------------------------------------ */
/* samplers and exhaustive enumeration                                      */
/* ------------------------------------------------------------------------ */

void or_sample_path(const or_graph *g, uint64_t seed, uint64_t first, uint64_t k, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    if (g->R_tau == 0)
        return;
    for (uint64_t i = 0; i < k; i++) {
        uint64_t r = or_draw(seed, 0u, first + i, g->R_tau);
        int32_t q[4];
        or_decode_path(g, r, q);
        tally[or_classify_path(g, q)]++;
    }
}

void or_sample_centered(const or_graph *g, uint64_t seed, uint64_t first, uint64_t k, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    if (g->R_lam == 0)
        return;
    for (uint64_t i = 0; i < k; i++) {
        uint64_t r = or_draw(seed, 1u, first + i, g->R_lam);
        int32_t q[4];
        or_decode_centered(g, r, q);
        tally[or_classify_centered(g, q)]++;
    }
}

void or_enumerate_path(const or_graph *g, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    for (uint64_t r = 0; r < g->R_tau; r++) {
        int32_t q[4];
        or_decode_path(g, r, q);
        tally[or_classify_path(g, q)]++;
    }
}

void or_enumerate_centered(const or_graph *g, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    for (uint64_t r = 0; r < g->R_lam; r++) {
        int32_t q[4];
        or_decode_centered(g, r, q);
        tally[or_classify_centered(g, q)]++;
    }
}
