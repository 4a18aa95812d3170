/*
 * Exact induced 4-vertex subgraph counts: the ground truth the sampling
 * oracle's estimates are judged against.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Two independent routes:
 *  - or_exact_brute: the definition itself.  Every 4-subset, its induced
 *    degree sequence, the motif it names (Section 2, Figure 1 numbering).
 *  - or_exact_formula: the split the paper describes for its enumeration
 *    code (Section 6): subgraph (non-induced) counts N_1..N_6, the three
 *    cycle-based ones by enumeration under a vertex ordering, the rest by
 *    direct formulas, then Eq. 1 (A C = N) solved by back-substitution.
 *      N_1 = sum_v C(d_v,3)                     3-stars
 *      N_2 = W - 3T, W = sum_e (d_u-1)(d_v-1)   3-paths
 *      N_3 = sum_v t_v (d_v - 2)                tailed triangles
 *      N_4 = #4-cycles (as subgraphs)           wedge pairs, max-vertex rule
 *      N_5 = sum_e C(t_e, 2)                    diamonds
 *      N_6 = #4-cliques
 *    t_v / t_e are the triangles on a vertex / an edge, T the triangles.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

int or_exact_brute(int64_t n, const int64_t *off, const int32_t *col, uint64_t C[7], uint64_t *T)
{
    int st = or_validate(n, off, col);
    if (st != OR_OK)
        return st;
    if (n > 512)
        return OR_EINVAL;
    unsigned char *adj = calloc((size_t)(n > 0 ? n * n : 1), 1);
    if (!adj)
        return OR_ENOMEM;
    for (int64_t v = 0; v < n; v++)
        for (int64_t s = off[v]; s < off[v + 1]; s++)
            adj[v * n + col[s]] = 1;
    uint64_t cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    uint64_t tri = 0;
    for (int64_t a = 0; a < n; a++)
        for (int64_t b = a + 1; b < n; b++)
            for (int64_t c = b + 1; c < n; c++) {
                int ab = adj[a * n + b], ac = adj[a * n + c], bc = adj[b * n + c];
                tri += (uint64_t)(ab && ac && bc);
                for (int64_t d = c + 1; d < n; d++) {
                    int ad = adj[a * n + d], bd = adj[b * n + d], cd = adj[c * n + d];
                    int deg[4] = {ab + ac + ad, ab + bc + bd, ac + bc + cd, ad + bd + cd};
                    /* sorted degree sequence -> motif; unconnected sets -> 0 */
                    for (int i = 0; i < 4; i++)
                        for (int j = i; j > 0 && deg[j - 1] > deg[j]; j--) {
                            int t = deg[j];
                            deg[j] = deg[j - 1];
                            deg[j - 1] = t;
                        }
                    int key = deg[0] * 1000 + deg[1] * 100 + deg[2] * 10 + deg[3];
                    int m = key == 1113 ? 1 : key == 1122 ? 2 : key == 1223 ? 3
                          : key == 2222 ? 4 : key == 2233 ? 5 : key == 3333 ? 6 : 0;
                    cnt[m]++;
                }
            }
    free(adj);
    C[0] = 0;
    for (int i = 1; i <= 6; i++)
        C[i] = cnt[i];
    *T = tri;
    return OR_OK;
}

/* ---- formula counter ----------------------------------------------------- */

static _Thread_local const int64_t *g_ex_off; /* per thread, like the relabel sort */

static int cmp_deg_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    int64_t da = g_ex_off[a + 1] - g_ex_off[a], db = g_ex_off[b + 1] - g_ex_off[b];
    if (da != db)
        return da < db ? -1 : 1;
    return (a > b) - (a < b);
}

int or_exact_formula(int64_t n, const int64_t *off, const int32_t *col, uint64_t C[7], uint64_t *T)
{
    int st = or_validate(n, off, col);
    if (st != OR_OK)
        return st;
    int64_t slots = off[n];
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *order = malloc(sizeof(int32_t) * nn);
    int32_t *rk = malloc(sizeof(int32_t) * nn);
    int64_t *foff = malloc(sizeof(int64_t) * (nn + 1));
    int32_t *fcol = malloc(sizeof(int32_t) * (size_t)(slots / 2 + 1));
    uint64_t *t_e = calloc((size_t)(slots / 2 + 1), sizeof(uint64_t));
    uint64_t *t_v = calloc(nn, sizeof(uint64_t));
    int64_t *mark = malloc(sizeof(int64_t) * nn);   /* slot+1 in N+(u), stamped */
    int32_t *stamp = malloc(sizeof(int32_t) * nn);
    int32_t *stamp2 = malloc(sizeof(int32_t) * nn);
    int64_t *cnt = calloc(nn, sizeof(int64_t));
    int32_t *touched = malloc(sizeof(int32_t) * nn);
    int32_t *common = malloc(sizeof(int32_t) * nn);
    if (!order || !rk || !foff || !fcol || !t_e || !t_v || !mark || !stamp || !stamp2 || !cnt ||
        !touched || !common) {
        st = OR_ENOMEM;
        goto done;
    }

    /* vertex ordering by (degree, id) */
    for (int64_t v = 0; v < n; v++)
        order[v] = (int32_t)v;
    g_ex_off = off;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_deg_id);
    for (int64_t i = 0; i < n; i++)
        rk[order[i]] = (int32_t)i;

    /* forward adjacency N+(u): neighbours of higher rank (input id order) */
    foff[0] = 0;
    for (int64_t u = 0; u < n; u++) {
        int64_t c = foff[u];
        for (int64_t s = off[u]; s < off[u + 1]; s++)
            if (rk[col[s]] > rk[u])
                fcol[c++] = col[s];
        foff[u + 1] = c;
    }

    /* triangles: each found once from its lowest-ranked vertex u */
    u128 tri = 0, k4 = 0;
    for (int64_t v = 0; v < n; v++) {
        stamp[v] = -1;
        stamp2[v] = -1;
    }
    for (int64_t u = 0; u < n; u++) {
        for (int64_t s = foff[u]; s < foff[u + 1]; s++) {
            stamp[fcol[s]] = (int32_t)u;
            mark[fcol[s]] = s;
        }
        for (int64_t s = foff[u]; s < foff[u + 1]; s++) {
            int32_t v = fcol[s];
            int64_t nc = 0;
            for (int64_t s2 = foff[v]; s2 < foff[v + 1]; s2++) {
                int32_t w = fcol[s2];
                if (stamp[w] == u) { /* triangle u, v, w */
                    tri++;
                    t_v[u]++;
                    t_v[v]++;
                    t_v[w]++;
                    t_e[s]++;        /* edge (u,v) */
                    t_e[s2]++;       /* edge (v,w) */
                    t_e[mark[w]]++;  /* edge (u,w) */
                    common[nc++] = w;
                }
            }
            /* 4-cliques u < v < w < x: x in N+(u), N+(v) and N+(w) */
            for (int64_t i = 0; i < nc; i++)
                stamp2[common[i]] = v;
            for (int64_t i = 0; i < nc; i++) {
                int32_t w = common[i];
                for (int64_t s3 = foff[w]; s3 < foff[w + 1]; s3++)
                    if (stamp2[fcol[s3]] == v)
                        k4++;
            }
            for (int64_t i = 0; i < nc; i++)
                stamp2[common[i]] = -1;
        }
    }

    /* 4-cycles (as subgraphs): for the highest-ranked vertex x of a cycle,
     * the opposite vertex y and the two middles w, w' are all lower; count
     * pairs of lower-ranked wedge middles between x and each lower y. */
    u128 n4 = 0;
    for (int64_t x = 0; x < n; x++) {
        int64_t nt = 0;
        for (int64_t s = off[x]; s < off[x + 1]; s++) {
            int32_t w = col[s];
            if (rk[w] >= rk[x])
                continue;
            for (int64_t s2 = off[w]; s2 < off[w + 1]; s2++) {
                int32_t y = col[s2];
                if (rk[y] >= rk[x])
                    continue;
                if (cnt[y] == 0)
                    touched[nt++] = y;
                cnt[y]++;
            }
        }
        for (int64_t i = 0; i < nt; i++) {
            u128 c = (u128)cnt[touched[i]];
            n4 += c * (c - 1) / 2;
            cnt[touched[i]] = 0;
        }
    }

    u128 n1 = 0, w = 0, n3 = 0, n5 = 0;
    for (int64_t v = 0; v < n; v++) {
        u128 d = (u128)(off[v + 1] - off[v]);
        if (d >= 3)
            n1 += d * (d - 1) * (d - 2) / 6;
        if (d >= 2)
            n3 += (u128)t_v[v] * (d - 2);
        for (int64_t s = off[v]; s < off[v + 1]; s++) {
            int32_t u2 = col[s];
            if (u2 < v)
                continue; /* each undirected edge once */
            u128 du2 = (u128)(off[u2 + 1] - off[u2]);
            w += (d - 1) * (du2 - 1);
        }
    }
    for (int64_t e = 0; e < foff[n]; e++) {
        u128 t = (u128)t_e[e];
        if (t >= 2)
            n5 += t * (t - 1) / 2;
    }
    i128 N1 = (i128)n1, N2 = (i128)w - 3 * (i128)tri, N3 = (i128)n3, N4 = (i128)n4, N5 = (i128)n5,
         N6 = (i128)k4;

    /* Eq. 1 is upper triangular with unit diagonal: solve from the bottom. */
    i128 c6 = N6;
    i128 c5 = N5 - 6 * c6;
    i128 c4 = N4 - 1 * c5 - 3 * c6;
    i128 c3 = N3 - 4 * c5 - 12 * c6;
    i128 c2 = N2 - 2 * c3 - 4 * c4 - 6 * c5 - 12 * c6;
    i128 c1 = N1 - 1 * c3 - 2 * c5 - 4 * c6;
    i128 cs[7] = {0, c1, c2, c3, c4, c5, c6};
    C[0] = 0;
    for (int i = 1; i <= 6; i++) {
        if (cs[i] < 0 || cs[i] >= ((i128)1 << 64)) {
            st = OR_EOVERFLOW;
            goto done;
        }
        C[i] = (uint64_t)cs[i];
    }
    *T = (uint64_t)tri;
    st = OR_OK;
done:
    free(order);
    free(rk);
    free(foff);
    free(fcol);
    free(t_e);
    free(t_v);
    free(mark);
    free(stamp);
    free(stamp2);
    free(cnt);
    free(touched);
    free(common);
    return st;
}
