/*
 * Alias-table variant of the weighted edge pick (Algorithm 1 step 2,
 * Algorithm 3 step 2): Walker's alias method, O(1) work per draw.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of the oracle: the checker of the
 * HIP library's alias draw, never a fallback for it.
 *
 * Exact integer table.  N slots with weights w[s] (total R, 0 < R < 2^64)
 * get N buckets of capacity R, and slot s owns mass N*w[s] of the N*R total.
 * Bucket b keeps K[b] <= R of slot b's own mass and holds R - K[b] of slot
 * alias[b]'s.  A draw takes b uniform in [0, N) and x uniform in [0, R) and
 * picks b if x < K[b], else alias[b]; slot s is then picked with probability
 *     (K[s] + sum over b with alias[b] = s, K[b] < R of (R - K[b])) / (N R)
 * which the construction makes exactly w[s] / R.
 *
 * Construction (one fixed table for given weights): Walker's sweep with both
 * lists in index order.  Light slots (N w < R) are visited in index order;
 * each keeps its whole mass and fills the rest of its bucket from the current
 * heavy slot (N w >= R, also in index order).  A heavy slot whose remaining
 * mass drops below R becomes a bucket itself: it keeps that remainder and
 * fills the rest from the next heavy slot.  Heavy slots never drawn below R
 * keep a full bucket (K = R, alias = itself).
 *
 * Random stream of one alias draw (the paper leaves the generator open; the
 * main samplers' Philox stream is extended): the candidate 64-bit words of
 * sample `id` in order -- words 0,1 then 2,3 of the Philox4x32-10 block with
 * counter (id, tag, attempt) for attempt 0, 1, ... -- where each bounded draw
 * takes candidates until Lemire's method accepts one and the next draw goes
 * on after it.  Three draws: b in [0, N), x in [0, R), then the position o in
 * [0, w[s]) inside the picked slot.  r = P[s-1] + o is then uniform on [0, R)
 * and decodes exactly as the main samplers' r.  Tags 2 (3-path) and 3
 * (centered) keep these streams apart from the main samplers' tags 0 and 1.
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

typedef unsigned __int128 u128;

static int64_t next_heavy(const uint64_t *w, int64_t N, u128 cap, int64_t from)
{
    for (int64_t s = from; s < N; s++)
        if ((u128)N * w[s] >= cap)
            return s;
    return -1;
}

int or_alias_build(const uint64_t *w, int64_t N, uint64_t *K, int64_t *alias)
{
    if (N <= 0 || !w || !K || !alias)
        return OR_EINVAL;
    u128 R = 0;
    for (int64_t s = 0; s < N; s++)
        R += w[s];
    if (R == 0 || R >= (((u128)1) << 64))
        return OR_EINVAL;
    const u128 cap = R;
    int64_t h = next_heavy(w, N, cap, 0); /* exists: the masses average R */
    if (h < 0)
        return OR_EINVAL;
    u128 resid = (u128)N * w[h]; /* mass of heavy h not yet given away */
    for (int64_t s = 0; s < N; s++) {
        const u128 M = (u128)N * w[s];
        if (M >= cap)
            continue; /* heavy: handled through h */
        K[s] = (uint64_t)M;
        alias[s] = h;
        resid -= cap - M; /* resid >= cap before, and the deficit is <= cap */
        while (resid < cap) {
            const int64_t hn = next_heavy(w, N, cap, h + 1);
            if (hn < 0)
                return OR_EINVAL; /* impossible when the masses sum to N R */
            K[h] = (uint64_t)resid;
            alias[h] = hn;
            resid = (u128)N * w[hn] - (cap - resid);
            h = hn;
        }
    }
    /* the current heavy slot and every later one keep a full bucket; the
     * mass balance leaves exactly R with each */
    if (resid != cap)
        return OR_EINVAL;
    for (int64_t s = h; s < N; s++) {
        const u128 M = (u128)N * w[s];
        if (M < cap)
            continue;
        if (s > h && M != cap)
            return OR_EINVAL;
        K[s] = (uint64_t)cap;
        alias[s] = s;
    }
    return OR_OK;
}

typedef struct {
    uint32_t key[2];
    uint32_t id_lo, id_hi, tag, attempt;
    uint32_t w[4];
    int next; /* next candidate word pair of w (2: a new block is due) */
} or_stream;

static void stream_init(or_stream *st, uint64_t seed, uint32_t tag, uint64_t id)
{
    st->key[0] = (uint32_t)seed;
    st->key[1] = (uint32_t)(seed >> 32);
    st->id_lo = (uint32_t)id;
    st->id_hi = (uint32_t)(id >> 32);
    st->tag = tag;
    st->attempt = 0;
    st->next = 2;
}

/* next accepted bounded draw in [0, R) from the stream (R >= 1) */
static uint64_t stream_bounded(or_stream *st, uint64_t R)
{
    for (;;) {
        if (st->next == 2) {
            const uint32_t ctr[4] = {st->id_lo, st->id_hi, st->tag, st->attempt};
            or_philox4x32_10(ctr, st->key, st->w);
            st->attempt++;
            st->next = 0;
        }
        const uint64_t x = (uint64_t)st->w[2 * st->next] | ((uint64_t)st->w[2 * st->next + 1] << 32);
        st->next++;
        uint64_t r;
        if (or_lemire(x, R, 64, &r))
            return r;
    }
}

uint64_t or_draw_alias(const uint64_t *P, const uint64_t *K, const int64_t *alias, int64_t N, uint64_t R,
                       uint64_t seed, uint32_t tag, uint64_t id)
{
    or_stream st;
    stream_init(&st, seed, tag, id);
    const uint64_t b = stream_bounded(&st, (uint64_t)N);
    const uint64_t x = stream_bounded(&st, R);
    const int64_t s = x < K[b] ? (int64_t)b : alias[b];
    const uint64_t below = s > 0 ? P[s - 1] : 0;
    const uint64_t o = stream_bounded(&st, P[s] - below);
    return below + o;
}

void or_sample_path_alias(const or_graph *g, const uint64_t *K, const int64_t *alias, uint64_t seed, uint64_t first,
                          uint64_t k, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    if (g->R_tau == 0)
        return;
    for (uint64_t i = 0; i < k; i++) {
        const uint64_t r = or_draw_alias(g->p_tau, K, alias, g->slots, g->R_tau, seed, 2u, first + i);
        int32_t q[4];
        or_decode_path(g, r, q);
        tally[or_classify_path(g, q)]++;
    }
}

void or_sample_centered_alias(const or_graph *g, const uint64_t *K, const int64_t *alias, uint64_t seed,
                              uint64_t first, uint64_t k, uint64_t tally[8])
{
    memset(tally, 0, 8 * sizeof(uint64_t));
    if (g->R_lam == 0)
        return;
    for (uint64_t i = 0; i < k; i++) {
        const uint64_t r = or_draw_alias(g->p_lam, K, alias, g->slots, g->R_lam, seed, 3u, first + i);
        int32_t q[4];
        or_decode_centered(g, r, q);
        tally[or_classify_centered(g, q)]++;
    }
}
