// Single-pass inclusive scan with decoupled look-back (Merrill & Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016), laid
// out for 64-wide wavefronts: each 256-thread block owns a tile of
// 256 * ITEMS consecutive elements, each wave a contiguous quarter of it,
// processed as ITEMS coalesced 64-element rows.  No LDS transposes: a wave
// first reduces its rows, wave 0 resolves the tile prefix by look-back, then
// every wave rescans its rows from registers and hands (index, inclusive
// value, element) to the output functor.
//
// In:  T operator()(int64_t i) const           element i (i < N)
// Out: void operator()(int64_t i, T incl, T x) inclusive prefix of element i
// Op:  associative and commutative (sum, max).
#pragma once

#include "common.hpp"

namespace pm {

template <typename T>
struct ScanState {
    T *agg;          // per-tile aggregate
    T *incl;         // per-tile inclusive prefix
    uint32_t *flag;  // 0 empty, 1 aggregate ready, 2 prefix ready
    uint32_t *ticket;
};

template <typename T>
struct SumOp {
    __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};

template <typename T>
struct MaxOp {
    __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
};

template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int d)
{
    return __shfl_up(v, d, kWave);
}

template <typename T>
__device__ __forceinline__ T shfl_t(T v, int src)
{
    return __shfl(v, src, kWave);
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_inclusive(T v, Op op, T identity)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = shfl_up_t(v, d);
        v = op(v, lane >= d ? o : identity);
    }
    return v;
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, Op op)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = op(v, __shfl_xor(v, d, kWave));
    return v;
}

template <typename T, int ITEMS, typename Op, typename In, typename Out>
__global__ __launch_bounds__(kBlock) void scan_kernel(In in, Out out, int64_t N, Op op, T identity,
                                                      ScanState<T> st)
{
    __shared__ uint32_t s_tile;
    __shared__ T s_wave[kBlock / kWave];
    __shared__ T s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(st.ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t wave_base = tile * (int64_t)(kBlock * ITEMS) + (int64_t)w * kWave * ITEMS;

    T v[ITEMS];
    T wsum = identity;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = wave_base + (int64_t)i * kWave + lane;
        v[i] = idx < N ? in(idx) : identity;
        wsum = op(wsum, v[i]);
    }
    wsum = wave_reduce(wsum, op);
    if (lane == 0) s_wave[w] = wsum;
    __syncthreads();

    if (w == 0) {
        T agg = identity;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) agg = op(agg, s_wave[i]);
        T excl = identity;
        if (tile == 0) {
            if (lane == 0) {
                st.incl[0] = agg;
                __hip_atomic_store(&st.flag[0], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            if (lane == 0) {
                st.agg[tile] = agg;
                __hip_atomic_store(&st.flag[tile], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            int64_t j = tile - 1;
            while (true) {
                const int64_t t = j - lane;
                uint32_t f = 2u;
                T val = identity;
                if (t >= 0) {
                    do {
                        f = __hip_atomic_load(&st.flag[t], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    } while (f == 0u);
                    val = (f == 2u) ? st.incl[t] : st.agg[t];
                }
                const uint64_t pmask = __ballot(f == 2u);
                const int first_p = pmask ? __builtin_ctzll(pmask) : kWave;
                T contrib = lane <= first_p ? val : identity;
                excl = op(excl, wave_reduce(contrib, op));
                if (pmask) break;
                j -= kWave;
            }
            if (lane == 0) {
                st.incl[tile] = op(excl, agg);
                __hip_atomic_store(&st.flag[tile], 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (lane == 0) s_prefix = excl;
    }
    __syncthreads();

    T run = s_prefix;
    for (int i = 0; i < w; ++i) run = op(run, s_wave[i]);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        T sc = wave_inclusive(v[i], op, identity);
        int64_t idx = wave_base + (int64_t)i * kWave + lane;
        if (idx < N) out(idx, op(run, sc), v[i]);
        run = op(run, shfl_t(sc, kWave - 1));
    }
}

// Scratch for one scan of N elements (tiles of 256 * ITEMS).
template <typename T>
struct ScanScratch {
    int64_t tiles = 0;
    size_t bytes = 0;
    static size_t bytes_for(int64_t N, int items)
    {
        int64_t tiles = (N + (int64_t)kBlock * items - 1) / ((int64_t)kBlock * items);
        if (tiles < 1) tiles = 1;
        return (size_t)tiles * (2 * sizeof(T) + sizeof(uint32_t)) + 256;
    }
};

// Launch a scan; `scratch` must hold ScanScratch<T>::bytes_for(N, ITEMS) bytes.
template <typename T, int ITEMS, typename Op, typename In, typename Out>
pm_status scan_launch(In in, Out out, int64_t N, Op op, T identity, void *scratch, hipStream_t s)
{
    if (N <= 0) return PM_OK;
    const int64_t tiles = (N + (int64_t)kBlock * ITEMS - 1) / ((int64_t)kBlock * ITEMS);
    char *p = (char *)scratch;
    ScanState<T> st;
    st.agg = (T *)p;
    p += tiles * sizeof(T);
    st.incl = (T *)p;
    p += tiles * sizeof(T);
    st.flag = (uint32_t *)p;
    st.ticket = st.flag + tiles;
    PM_TRY(fill_async<uint32_t>(st.flag, 0u, tiles + 1, s));
    hipLaunchKernelGGL((scan_kernel<T, ITEMS, Op, In, Out>), dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, N,
                       op, identity, st);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
