// The sampling kernels: Algorithm 1 (sample) classified as in Algorithm 2,
// and Algorithm 3 (sample-centered) classified as in Algorithm 4.
//
// One lane per sample, grid-stride over sample ids.  Per sample:
//   r      exact uniform in [0, R) from Philox keyed by (seed, id)
//   slot   first s with P[s] > r: guide table, then a short binary search
//   picks  o = r - P[s-1] split in mixed radix into the two neighbour picks
//   tests  the three adjacency tests by binary search in the shorter row
//          (after the relabel, the smaller id has the shorter or equal row)
//   tally  per-lane counters, one wave reduction and atomic per class
#include "graph.hpp"
#include "profile.hpp"

#include <algorithm>
#include <mutex>

namespace pm {

// b in row a?  Searches the row of the smaller id.
__device__ __forceinline__ uint32_t adjacent(const int64_t *__restrict__ off, const uint32_t *__restrict__ col,
                                             uint32_t a, uint32_t b)
{
    const uint32_t x = a < b ? a : b, y = a < b ? b : a;
    int64_t lo = off[x];
    const int64_t end = off[x + 1];
    int64_t hi = end;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < y)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < end && col[lo] == y) ? 1u : 0u;
}

template <bool CENTERED>
__global__ __launch_bounds__(kBlock) void k_sample(SamplerView g, uint64_t seed, uint64_t first, uint64_t k,
                                                   unsigned long long *__restrict__ tally)
{
    uint32_t cnt[PM_NUM_TALLIES];
#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] = 0;

    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
        const uint64_t r = draw_bounded(seed, CENTERED ? 1u : 0u, first + i, g.R);

        // edge draw: s = min{s : P[s] > r}
        const uint64_t j = r >> g.shift;
        uint32_t lo = g.guide[j], hi = g.guide[j + 1];
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (g.P[mid] > r)
                hi = mid;
            else
                lo = mid + 1;
        }
        const uint32_t s = lo;
        const uint32_t u = g.src[s], v = g.col[s];
        const uint64_t below = s ? g.P[s - 1] : 0ull;
        const uint64_t o = r - below;
        const int64_t ou = g.off[u], du = g.off[u + 1] - ou;
        const int64_t ov = g.off[v], dv = g.off[v + 1] - ov;

        uint32_t up, vp;
        if (!CENTERED) {
            // o in [0, (d_u-1)(d_v-1)): u' is the a-th of N(u)\{v}, v' the b-th of N(v)\{u}
            uint64_t a, b;
            divmod_small(o, (uint32_t)(dv - 1), a, b);
            up = g.col[ou + (int64_t)a];
            if (up == v) up = g.col[ou + du - 1];
            vp = g.col[ov + (int64_t)b];
            if (vp == u) vp = g.col[ov + dv - 1];
        } else {
            // o in [0, L_uv L_vu): u' among the L_uv neighbours of u after v,
            // v' among the L_vu neighbours of v after u (row suffixes)
            const uint64_t lam = g.P[s] - below;
            const uint32_t luv = (uint32_t)(du - 1 - ((int64_t)s - ou));
            uint64_t lvu, rem, a, b;
            divmod_small(lam, luv, lvu, rem);
            divmod_small(o, (uint32_t)lvu, a, b);
            up = g.col[(int64_t)s + 1 + (int64_t)a];
            vp = g.col[ov + (dv - (int64_t)lvu) + (int64_t)b];
        }

        uint32_t cls;
        if (up == vp) {
            cls = PM_TALLY_TRI;
        } else if (!CENTERED) {
            const uint32_t x = adjacent(g.off, g.col, up, v);
            const uint32_t y = adjacent(g.off, g.col, u, vp);
            const uint32_t z = adjacent(g.off, g.col, up, vp);
            const uint32_t e = x + y + z;
            // 3 edges: 3-path; 4: 4-cycle if the closing edge, else tailed
            // triangle; 5: chordal-4-cycle; 6: 4-clique
            cls = e == 0 ? 2u : e == 1 ? (z ? 4u : 3u) : e == 2 ? 5u : 6u;
        } else {
            if (!adjacent(g.off, g.col, up, vp)) {
                cls = PM_TALLY_OPEN;
            } else {
                cls = 4u + adjacent(g.off, g.col, up, v) + adjacent(g.off, g.col, u, vp);
            }
        }
#pragma unroll
        for (int c = 0; c < PM_NUM_TALLIES; ++c) cnt[c] += (cls == (uint32_t)c);
    }

#pragma unroll
    for (int c = 0; c < PM_NUM_TALLIES; ++c) {
        uint32_t t = wave_sum_u32(cnt[c]);
        if (lane_id() == 0 && t) atomicAdd(&tally[c], (unsigned long long)t);
    }
}

static int cu_count(int dev)
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

static pm_status launch_sampler(const pm_graph *g, bool centered, uint64_t seed, uint64_t first, uint64_t k,
                                uint64_t *tally, hipStream_t s)
{
    const SamplerView v = view_of(g, centered);
    if (v.R == 0 || k == 0) return PM_OK;
    const uint64_t want = (k + kBlock - 1) / kBlock;
    const uint64_t cap = (uint64_t)cu_count(g->device) * 16;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min(want, cap));
    ProfScope prof(centered ? "sample_centered" : "sample_path", s);
    if (centered)
        hipLaunchKernelGGL(k_sample<true>, dim3(blocks), dim3(kBlock), 0, s, v, seed, first, k,
                           (unsigned long long *)tally);
    else
        hipLaunchKernelGGL(k_sample<false>, dim3(blocks), dim3(kBlock), 0, s, v, seed, first, k,
                           (unsigned long long *)tally);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

pm_status check_device(const pm_graph *g);

pm_status sample_async(const pm_graph *g, const pm_params *p, uint64_t *tallies_dev, hipStream_t s)
{
    if (!g || !p || !tallies_dev) {
        set_error("null argument");
        return PM_EINVAL;
    }
    PM_TRY(check_device(g));
    PM_TRY(fill_async<uint64_t>(tallies_dev, 0ull, 2 * PM_NUM_TALLIES, s));
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

pm_status count_on_graph(const pm_graph *g, const pm_params *p, pm_result *out, hipStream_t s)
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
    pm_status st = sample_async(g, p, t, s);
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

}  // namespace pm
