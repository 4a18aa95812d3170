// Alias-table variant of the weighted edge pick (Algorithm 1 step 2,
// Algorithm 3 step 2): Walker's alias method, one table line per draw
// instead of a guide entry and a search over the prefix array.
//
// Table (exact, integer).  N slots with weights w_s and total R get N buckets
// of capacity R; slot s owns mass M_s = N w_s of the N R total.  Bucket b
// keeps K_b <= R of its own slot's mass and holds R - K_b of slot alias_b's.
// A draw takes b uniform in [0, N), x uniform in [0, R), picks b if x < K_b
// and alias_b otherwise: slot s comes up with probability w_s / R exactly.
//
// Which table: Walker's sweep with both lists in index order (light slots,
// M < R, each filling its bucket from the current heavy slot, M >= R; a heavy
// slot drawn below R becoming a bucket filled from the next heavy slot).  In
// closed form, with D_i the deficits R - M of the first i light slots and E_h
// the excesses M - R of heavy slots 0..h (both prefix sums, 128-bit):
//   light slot i:  K = M, alias = heavy slot #{h : E_h < D_i}
//   heavy slot h:  K = R + E_h - (first D_i above E_h), alias = heavy h + 1,
//                  or K = R (alias itself) when no D_i lies above E_h
// Both counts come from one merge of the D and E sequences (ties: D first),
// done here with merge-path tiles; the whole build is scans, one merge and
// streaming passes.
//
// Draw stream: the sample's Philox candidates (words 0,1 then 2,3 of the
// block with counter (id, tag, attempt), attempts 0, 1, ...) taken in order
// by three bounded draws: b in [0, N), x in [0, R), then the position o in
// [0, w_s) inside the picked slot.  Tags 2 (3-path) and 3 (centered).  The
// sample is then decoded from (s, o) exactly as the main samplers decode it.
#include "graph.hpp"
#include "profile.hpp"
#include "drawsort.hpp"
#include "sampler.hpp"
#include "scan.hpp"
#include "streams.hpp"

#include <algorithm>
#include <mutex>
#include <vector>

namespace pm {

pm_status check_device(const pm_graph *g);
int sampler_cu_count(int dev);
pm_status count_with(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s,
                     pm_status (*run)(const pm_graph *, const pm_params *, uint64_t *, hipStream_t));

namespace {

// 128-bit sums and comparisons on (lo, hi) pairs
struct U128SumOp {
    __device__ __forceinline__ U64x2 operator()(U64x2 x, U64x2 y) const
    {
        const uint64_t lo = x.a + y.a;
        return U64x2{lo, x.b + y.b + (lo < x.a ? 1ull : 0ull)};
    }
};

__device__ __forceinline__ bool le128(U64x2 x, U64x2 y) { return x.b < y.b || (x.b == y.b && x.a <= y.a); }

// weight of slot s from the per-segment prefix (it restarts at each segment)
__device__ __forceinline__ uint64_t weight_of(const uint64_t *__restrict__ P, int64_t s)
{
    return P[s] - ((s & (kPrefixSeg - 1)) ? P[s - 1] : 0ull);
}

// M = N w in 128 bits
__device__ __forceinline__ U64x2 mass_of(uint64_t w, uint64_t N) { return U64x2{w * N, __umul64hi(w, N)}; }

__device__ __forceinline__ bool is_light(uint64_t w, uint64_t N, uint64_t R)
{
    const U64x2 m = mass_of(w, N);
    return m.b == 0 && m.a < R;
}

// light flags -> light rank of every slot, and the light / heavy slot lists
struct LightIn {
    const uint64_t *P;
    uint64_t N, R;
    __device__ __forceinline__ uint32_t operator()(int64_t i) const { return is_light(weight_of(P, i), N, R) ? 1u : 0u; }
};
struct ListOut {
    uint32_t *lpos, *L, *H;
    __device__ __forceinline__ void operator()(int64_t i, uint32_t incl, uint32_t x) const
    {
        const uint32_t ex = incl - x;
        lpos[i] = ex;
        if (x)
            L[ex] = (uint32_t)i;
        else
            H[i - ex] = (uint32_t)i;
    }
};

// deficits R - M of the light slots, excesses M - R of the heavy slots
struct DeficitIn {
    const uint64_t *P;
    const uint32_t *L;
    uint64_t N, R;
    __device__ __forceinline__ U64x2 operator()(int64_t i) const
    {
        return U64x2{R - weight_of(P, L[i]) * N, 0ull};  // N w < R here
    }
};
struct ExcessIn {
    const uint64_t *P;
    const uint32_t *H;
    uint64_t N, R;
    __device__ __forceinline__ U64x2 operator()(int64_t i) const
    {
        const U64x2 m = mass_of(weight_of(P, H[i]), N);  // >= R here
        return U64x2{m.a - R, m.b - (m.a < R ? 1ull : 0ull)};
    }
};
struct Store128 {
    U64x2 *dst;
    __device__ __forceinline__ void operator()(int64_t i, U64x2 incl, U64x2) const { dst[i] = incl; }
};

constexpr int kMergePer = 16;                       // merged outputs per thread
constexpr int kMergeTile = kBlock * kMergePer;      // per block

// Merge order: D[i] before E[h] iff D[i] <= E[h].  Number of D elements among
// the first d of the merge (smallest i with D[i] > E[d - i - 1]).
__device__ __forceinline__ int64_t merge_split(const U64x2 *D, int64_t nl, const U64x2 *E, int64_t nh, int64_t d)
{
    int64_t lo = d > nh ? d - nh : 0, hi = d < nl ? d : nl;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (le128(D[mid], E[d - mid - 1]))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// split[t] = D elements before tile t of the merge (t = 0 .. ntiles)
__global__ void k_merge_split(const U64x2 *__restrict__ D, int64_t nl, const U64x2 *__restrict__ E, int64_t nh,
                              int64_t ntiles, uint32_t *__restrict__ split)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    const int64_t d = std::min<int64_t>(t * kMergeTile, nl + nh);
    split[t] = (uint32_t)merge_split(D, nl, E, nh, d);
}

// One merge tile per block, staged in LDS.  Emitting D[i] records cD[i] =
// E elements before it (= #{h : E_h < D_i}); emitting E[h] records the kept
// mass of heavy slot h from the next D element (or R when there is none).
__global__ __launch_bounds__(kBlock) void k_merge(const U64x2 *__restrict__ D, int64_t nl,
                                                  const U64x2 *__restrict__ E, int64_t nh,
                                                  const uint32_t *__restrict__ split, uint64_t R,
                                                  uint32_t *__restrict__ cD, uint64_t *__restrict__ Kh)
{
    __shared__ U64x2 s_v[kMergeTile + 1];
    const int64_t t = blockIdx.x;
    const int64_t d0 = t * kMergeTile, d1 = std::min<int64_t>(d0 + kMergeTile, nl + nh);
    const int64_t i0 = split[t], i1 = split[t + 1], h0 = d0 - i0, h1 = d1 - i1;
    const int nD = (int)(i1 - i0), nE = (int)(h1 - h0);
    const int nDx = nD + (i1 < nl ? 1 : 0);  // plus the first D after the tile
    for (int j = threadIdx.x; j < nDx; j += blockDim.x) s_v[j] = D[i0 + j];
    for (int j = threadIdx.x; j < nE; j += blockDim.x) s_v[nDx + j] = E[h0 + j];
    __syncthreads();
    const U64x2 *sD = s_v, *sE = s_v + nDx;
    const int dd = std::min((int)threadIdx.x * kMergePer, nD + nE), de = std::min(dd + kMergePer, nD + nE);
    int i = (int)merge_split(sD, nD, sE, nE, dd), h = dd - i;
    for (int q = dd; q < de; ++q) {
        if (i < nD && (h >= nE || le128(sD[i], sE[h]))) {
            cD[i0 + i] = (uint32_t)(h0 + h);
            ++i;
        } else {
            // the first D after E[h] is D[i0 + i] (in LDS up to index nD)
            uint64_t K = R;
            if (i0 + i < nl) {
                const U64x2 X = sD[i], Eh = sE[h];
                K = R - (X.a - Eh.a);  // X - E_h is in (0, R]: its low word suffices
            }
            Kh[h0 + h] = K;
            ++h;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_alias_fill(const uint64_t *__restrict__ P, int64_t N, uint64_t R,
                                                       const uint32_t *__restrict__ lpos,
                                                       const uint32_t *__restrict__ H, int64_t nh,
                                                       const uint32_t *__restrict__ cD,
                                                       const uint64_t *__restrict__ Kh, AliasEntry *__restrict__ T)
{
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N; s += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t w = weight_of(P, s);
        const uint32_t ex = lpos[s];
        uint64_t K;
        uint32_t a;
        if (is_light(w, (uint64_t)N, R)) {
            K = w * (uint64_t)N;
            const uint32_t c = ex == 0 ? 0u : cD[ex - 1];
            a = H[std::min<int64_t>(c, nh - 1)];  // c < nh: the excesses sum to the deficits
        } else {
            const int64_t h = s - ex;
            K = Kh[h];
            a = (K < R && h + 1 < nh) ? H[h + 1] : (uint32_t)s;
        }
        AliasEntry e;
        e.K = K;
        e.w_self = w;
        e.w_alias = weight_of(P, a);
        e.alias = a;
        e.pad = 0;
        T[s] = e;
    }
}

// The table of one sampler's weights (per-segment prefix P over N slots,
// total R > 0).
pm_status build_table(const uint64_t *P, int64_t N, uint64_t R, AliasEntry *T, hipStream_t s)
{
    Temps tmp(s);
    uint32_t *lpos, *L, *H;
    PM_TRY(tmp.get(&lpos, (size_t)N));
    PM_TRY(tmp.get(&L, (size_t)N));
    PM_TRY(tmp.get(&H, (size_t)N));
    {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<uint32_t>::bytes_for(N, 16)));
        PM_TRY((scan_launch<uint32_t, 16>(LightIn{P, (uint64_t)N, R}, ListOut{lpos, L, H}, N, SumOp<uint32_t>(), 0u,
                                          scr, s)));
    }
    uint32_t last_pos = 0;
    uint64_t tail[2] = {0, 0};
    PM_HIP(hipMemcpyAsync(&last_pos, lpos + N - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(tail + 1, P + N - 1, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    if (N > 1) PM_HIP(hipMemcpyAsync(tail, P + N - 2, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    const unsigned __int128 m_last = (unsigned __int128)(tail[1] - tail[0]) * (uint64_t)N;
    const int64_t nl = (int64_t)last_pos + (m_last < R ? 1 : 0), nh = N - nl;
    if (nh <= 0) {
        set_error("internal: alias table without a heavy slot");
        return PM_EDEVICE;
    }
    U64x2 *D = nullptr, *E = nullptr;
    PM_TRY(tmp.get(&D, (size_t)std::max<int64_t>(nl, 1)));
    PM_TRY(tmp.get(&E, (size_t)nh));
    {
        char *scr = nullptr;
        PM_TRY(tmp.get(&scr, ScanScratch<U64x2>::bytes_for(N, 8)));
        if (nl > 0)
            PM_TRY((scan_launch<U64x2, 8>(DeficitIn{P, L, (uint64_t)N, R}, Store128{D}, nl, U128SumOp(),
                                          U64x2{0, 0}, scr, s)));
        PM_TRY((scan_launch<U64x2, 8>(ExcessIn{P, H, (uint64_t)N, R}, Store128{E}, nh, U128SumOp(), U64x2{0, 0},
                                      scr, s)));
    }
    // the deficits and the excesses balance exactly
    U64x2 dl{0, 0}, el{0, 0};
    if (nl > 0) PM_HIP(hipMemcpyAsync(&dl, D + nl - 1, sizeof(U64x2), hipMemcpyDeviceToHost, s));
    PM_HIP(hipMemcpyAsync(&el, E + nh - 1, sizeof(U64x2), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (dl.a != el.a || dl.b != el.b) {
        set_error("internal: alias table deficits and excesses differ");
        return PM_EDEVICE;
    }
    uint32_t *cD = nullptr, *split = nullptr;
    uint64_t *Kh = nullptr;
    const int64_t ntiles = (N + kMergeTile - 1) / kMergeTile;
    PM_TRY(tmp.get(&cD, (size_t)std::max<int64_t>(nl, 1)));
    PM_TRY(tmp.get(&Kh, (size_t)nh));
    PM_TRY(tmp.get(&split, (size_t)(ntiles + 1)));
    {
        ProfScope pm_("alias.merge", s);
        hipLaunchKernelGGL(k_merge_split, dim3((unsigned)((ntiles + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           D, nl, E, nh, ntiles, split);
        hipLaunchKernelGGL(k_merge, dim3((unsigned)ntiles), dim3(kBlock), 0, s, D, nl, E, nh, split, R, cD, Kh);
        PM_HIP(hipGetLastError());
    }
    {
        ProfScope pf("alias.fill", s);
        hipLaunchKernelGGL(k_alias_fill, dim3(grid_for(N, kBlock, 1 << 22)), dim3(kBlock), 0, s, P, N, R, lpos, H,
                           nh, cD, Kh, T);
        PM_HIP(hipGetLastError());
    }
    PM_HIP(hipStreamSynchronize(s));  // the temporaries go back to the cache after this
    return PM_OK;
}

// The stream of candidate words of one sample (see the file comment).
struct DrawStream {
    uint32_t k0, k1, id_lo, id_hi, tag, attempt;
    U32x4 w;
    int next;
    __device__ __forceinline__ DrawStream(uint64_t seed, uint32_t tg, uint64_t id)
        : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), id_lo((uint32_t)id), id_hi((uint32_t)(id >> 32)), tag(tg),
          attempt(0), w{0, 0, 0, 0}, next(2)
    {
    }
    __device__ __forceinline__ uint64_t bounded(uint64_t R)
    {
        for (;;) {
            if (next == 2) {
                w = philox4x32_10(U32x4{id_lo, id_hi, tag, attempt}, k0, k1);
                ++attempt;
                next = 0;
            }
            const uint64_t x = next == 0 ? ((uint64_t)w.x | ((uint64_t)w.y << 32))
                                         : ((uint64_t)w.z | ((uint64_t)w.w << 32));
            ++next;
            bool ok;
            const uint64_t r = lemire_try(x, R, ok);
            if (ok) return r;
        }
    }
};

// one alias-drawn sample (the stream's three draws, then the usual decode)
template <bool CENTERED>
__device__ __forceinline__ uint32_t alias_sample(const SamplerView &g, const AliasEntry *__restrict__ T, uint64_t N,
                                                 uint64_t seed, uint64_t id)
{
    DrawStream st(seed, CENTERED ? 3u : 2u, id);
    const uint64_t b = st.bounded(N);
    const uint64_t x = st.bounded(g.R);
    const uint4 *q = reinterpret_cast<const uint4 *>(T + b);
    const uint4 e0 = q[0], e1 = q[1];
    const uint64_t K = (uint64_t)e0.x | ((uint64_t)e0.y << 32);
    const bool keep = x < K;
    const uint32_t s = keep ? (uint32_t)b : e1.z;
    const uint64_t ws = keep ? ((uint64_t)e0.z | ((uint64_t)e0.w << 32)) : ((uint64_t)e1.x | ((uint64_t)e1.y << 32));
    const uint64_t o = st.bounded(ws);
    return sample_decode<CENTERED>(g, s, o, ws);
}

template <bool CENTERED>
__global__ __launch_bounds__(kBlock) void k_sample_alias(SamplerView g, const AliasEntry *__restrict__ T, uint64_t N,
                                                         uint64_t seed, uint64_t first, uint64_t k,
                                                         unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += nthreads)
        tally_add(cnt, alias_sample<CENTERED>(g, T, N, seed, first + i));
    tally_flush(cnt, tally);
}

// Draw order for the alias draw: the key is the top bits of the bucket b (the
// stream's first draw), so neighbouring lanes read neighbouring table lines.
struct AliasKey {
    uint64_t N, seed, first;
    uint32_t tag;
    int kshift;
    __device__ uint32_t operator()(int64_t i) const
    {
        DrawStream st(seed, tag, first + (uint64_t)i);
        return (uint32_t)(st.bounded(N) >> kshift);
    }
};

template <bool CENTERED>
__global__ __launch_bounds__(kBlock) void k_sample_alias_sorted(SamplerView g, const AliasEntry *__restrict__ T,
                                                                uint64_t N, uint64_t seed, uint64_t first, uint64_t k,
                                                                const uint32_t *__restrict__ ids,
                                                                unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k; j += (uint64_t)gridDim.x * blockDim.x)
        tally_add(cnt, alias_sample<CENTERED>(g, T, N, seed, first + ids[j]));
    tally_flush(cnt, tally);
}

// Buffers of one alias draw-order sort chunk of min(k, kSortedChunk) ids.
pm_status alias_sort_bufs(Temps &tmp, uint64_t k, DrawSortBufs *b)
{
    const uint64_t chunk = std::min<uint64_t>(k, kSortedChunk);
    char *base = nullptr;
    PM_TRY(tmp.get(&base, draw_sort_bytes(chunk)));
    draw_sort_carve(base, chunk, b);
    return PM_OK;
}

// the ids [first, first + kc) sorted by their bucket keys (kc <= b.chunk);
// *ids receives the sorted ids (minus first)
pm_status alias_sort_chunk(uint64_t N, bool centered, uint64_t seed, uint64_t first, uint64_t kc, hipStream_t s,
                           const DrawSortBufs &b, uint32_t **ids)
{
    const int nbits = bits_for(N - 1);  // b < N
    const int kshift = nbits > kDrawKeyBits ? nbits - kDrawKeyBits : 0;
    const int kbits = nbits - kshift;
    return draw_sort("alias_draw_sort", AliasKey{N, seed, first, centered ? 3u : 2u, kshift}, kc, kbits, s, b, ids);
}

// the samples first + ids[j] for j < kc, into tally
pm_status alias_sample_chunk(const SamplerView &v, const AliasEntry *T, uint64_t N, bool centered, uint64_t seed,
                             uint64_t first, uint64_t kc, const uint32_t *ids, uint64_t *tally, unsigned blocks,
                             hipStream_t s)
{
    const unsigned kb = (unsigned)std::min<uint64_t>((kc + kBlock - 1) / kBlock, blocks);
    if (centered)
        hipLaunchKernelGGL((k_sample_alias_sorted<true>), dim3(kb), dim3(kBlock), 0, s, v, T, N, seed, first, kc, ids,
                           (unsigned long long *)tally);
    else
        hipLaunchKernelGGL((k_sample_alias_sorted<false>), dim3(kb), dim3(kBlock), 0, s, v, T, N, seed, first, kc,
                           ids, (unsigned long long *)tally);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

pm_status launch_alias_sorted(const SamplerView &v, const AliasEntry *T, uint64_t N, bool centered, uint64_t seed,
                              uint64_t first, uint64_t k, uint64_t *tally, unsigned blocks, hipStream_t s)
{
    Temps tmp(s);
    DrawSortBufs b{};
    PM_TRY(alias_sort_bufs(tmp, k, &b));
    for (uint64_t c0 = 0; c0 < k; c0 += b.chunk) {
        const uint64_t kc = std::min(b.chunk, k - c0);
        uint32_t *ids = nullptr;
        PM_TRY(alias_sort_chunk(N, centered, seed, first + c0, kc, s, b, &ids));
        PM_TRY(alias_sample_chunk(v, T, N, centered, seed, first + c0, kc, ids, tally, blocks, s));
    }
    return PM_OK;
}

pm_status launch_alias(const pm_graph *g, bool centered, uint64_t seed, uint64_t first, uint64_t k,
                       uint64_t *tally, hipStream_t s)
{
    const SamplerView v = view_of(g, centered);
    if (v.R == 0 || k == 0) return PM_OK;
    const AliasEntry *T = (const AliasEntry *)(centered ? g->alias_lam : g->alias_tau);
    const uint64_t want = (k + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)sampler_cu_count(g->device) * 4u;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
    const uint64_t N = (uint64_t)g->slots;
    ProfScope prof(centered ? "sample_centered_alias" : "sample_path_alias", s);
    if (k >= draw_order_min() && N > 1 && draw_order_enabled())
        return launch_alias_sorted(v, T, N, centered, seed, first, k, tally, (unsigned)cap, s);
    if (centered)
        hipLaunchKernelGGL((k_sample_alias<true>), dim3(blocks), dim3(kBlock), 0, s, v, T, N, seed, first, k,
                           (unsigned long long *)tally);
    else
        hipLaunchKernelGGL((k_sample_alias<false>), dim3(blocks), dim3(kBlock), 0, s, v, T, N, seed, first, k,
                           (unsigned long long *)tally);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

pm_status sample_alias_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, hipStream_t s)
{
    if ((g->R_tau && !g->alias_tau) || (g->R_lam && !g->alias_lam)) {
        set_error("alias draw: the graph has no alias tables (pm_graph_build_alias)");
        return PM_EINVAL;
    }
    PM_TRY(fill_async<uint64_t>(tallies_dev, 0ull, 2 * PM_NUM_TALLIES, s));
    const uint64_t N = (uint64_t)g->slots;
    const auto one_chunk = [&](uint64_t R, uint64_t k) {
        return R > 0 && k > 0 && k >= draw_order_min() && N > 1 && draw_order_enabled() && k <= kSortedChunk;
    };
    if (one_chunk(g->R_tau, p->k_path) && one_chunk(g->R_lam, p->k_cent)) {
        // as the main draw does: the centered sampler's ids sorted on a side
        // stream beside the 3-path sampler's sort, joined before the samples
        const SamplerView vp = view_of(g, false), vc = view_of(g, true);
        const AliasEntry *Tp = (const AliasEntry *)g->alias_tau, *Tc = (const AliasEntry *)g->alias_lam;
        const unsigned cap = (unsigned)((uint64_t)sampler_cu_count(g->device) * 4u);
        Temps tmp(s);
        DrawSortBufs bp{}, bc{};
        PM_TRY(alias_sort_bufs(tmp, p->k_path, &bp));
        PM_TRY(alias_sort_bufs(tmp, p->k_cent, &bc));
        hipStream_t side[2];
        PM_HIP(side_streams(side));
        uint32_t *ids_c = nullptr, *ids_p = nullptr;
        {
            Fork fork(s, side, 1);  // joined before the temporaries are released on s
            PM_HIP(fork.status);
            PM_TRY(alias_sort_chunk(N, true, p->seed, p->first_id_cent, p->k_cent, side[0], bc, &ids_c));
            PM_TRY(alias_sort_chunk(N, false, p->seed, p->first_id_path, p->k_path, s, bp, &ids_p));
            PM_HIP(fork.join());  // before the 3-path kernel, as the main draw does
        }
        {
            ProfScope prof("sample_path_alias", s);
            PM_TRY(alias_sample_chunk(vp, Tp, N, false, p->seed, p->first_id_path, p->k_path, ids_p, tallies_dev, cap,
                                      s));
        }
        ProfScope prof("sample_centered_alias", s);
        return alias_sample_chunk(vc, Tc, N, true, p->seed, p->first_id_cent, p->k_cent, ids_c,
                                  tallies_dev + PM_NUM_TALLIES, cap, s);
    }
    PM_TRY(launch_alias(g, false, p->seed, p->first_id_path, p->k_path, tallies_dev, s));
    PM_TRY(launch_alias(g, true, p->seed, p->first_id_cent, p->k_cent, tallies_dev + PM_NUM_TALLIES, s));
    return PM_OK;
}

std::mutex g_alias_mu;  // one table build per graph at a time

}  // namespace

pm_status graph_build_alias(pm_graph *g, hipStream_t s)
{
    if (!g) {
        set_error("null graph");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    std::lock_guard<std::mutex> lk(g_alias_mu);
    ProfScope prof("alias_build", s);
    for (int c = 0; c < 2; ++c) {
        void **slot = c ? &g->alias_lam : &g->alias_tau;
        const uint64_t R = c ? g->R_lam : g->R_tau;
        if (*slot || R == 0) continue;
        void *T = nullptr;
        PM_TRY(dev_alloc(&T, sizeof(AliasEntry) * (size_t)g->slots, s));
        const pm_status st = build_table(c ? g->p_lam : g->p_tau, g->slots, R, (AliasEntry *)T, s);
        if (st != PM_OK) {
            dev_free(T, s);
            return st;
        }
        *slot = T;
        g->bytes += sizeof(AliasEntry) * (uint64_t)g->slots;
    }
    return PM_OK;
}

pm_status graph_alias_export(const pm_graph *g, int32_t centered, uint64_t *K, int64_t *alias, hipStream_t s)
{
    if (!g || (g->slots > 0 && (!K || !alias))) {
        set_error("null argument");
        return PM_EINVAL;
    }
    const void *T = centered ? g->alias_lam : g->alias_tau;
    if (!T) {
        set_error("alias export: no table for this sampler (not built, or its total weight is 0)");
        return PM_EINVAL;
    }
    std::vector<AliasEntry> h((size_t)g->slots);
    PM_HIP(hipMemcpyAsync(h.data(), T, sizeof(AliasEntry) * h.size(), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < h.size(); ++i) {
        K[i] = h[i].K;
        alias[i] = h[i].alias;
    }
    return PM_OK;
}

pm_status count_alias(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s)
{
    return count_with(g, p, out, s, sample_alias_async);
}

}  // namespace pm
