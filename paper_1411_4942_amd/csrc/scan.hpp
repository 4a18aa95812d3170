// Inclusive scan in three launches (reduce, scan of tile sums, rescan),
// laid out for 64-wide wavefronts.  No block ever waits on another: each
// 256-thread block owns a tile of 256 * ITEMS consecutive elements, each wave
// a contiguous quarter of it processed as ITEMS coalesced 64-element rows.
//   1. every block reduces its tile                       -> tile_sums[tile]
//   2. one block turns tile_sums into exclusive prefixes (in place)
//   3. every block reloads its tile and rescans it from its prefix
// The input functor is evaluated twice (launches 1 and 3).
//
// In:  T operator()(int64_t i) const           element i (i < N)
// Out: void operator()(int64_t i, T incl, T x) inclusive prefix of element i
// Op:  associative and commutative (sum, max, pairwise sum).
#pragma once

#include "common.hpp"

namespace pm {

template <typename T>
struct SumOp {
    __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};

// a pair of 64-bit sums scanned together
struct U64x2 {
    uint64_t a, b;
};
struct PairSumOp {
    __device__ __forceinline__ U64x2 operator()(U64x2 x, U64x2 y) const { return U64x2{x.a + y.a, x.b + y.b}; }
};

template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int d)
{
    return __shfl_up(v, d, kWave);
}
template <typename T>
__device__ __forceinline__ T shfl_idx_t(T v, int src)
{
    return __shfl(v, src, kWave);
}
template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int m)
{
    return __shfl_xor(v, m, kWave);
}
template <>
__device__ __forceinline__ U64x2 shfl_up_t<U64x2>(U64x2 v, int d)
{
    return U64x2{__shfl_up(v.a, d, kWave), __shfl_up(v.b, d, kWave)};
}
template <>
__device__ __forceinline__ U64x2 shfl_idx_t<U64x2>(U64x2 v, int src)
{
    return U64x2{__shfl(v.a, src, kWave), __shfl(v.b, src, kWave)};
}
template <>
__device__ __forceinline__ U64x2 shfl_xor_t<U64x2>(U64x2 v, int m)
{
    return U64x2{__shfl_xor(v.a, m, kWave), __shfl_xor(v.b, m, kWave)};
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
    for (int d = kWave / 2; d > 0; d >>= 1) v = op(v, shfl_xor_t(v, d));
    return v;
}

template <typename T, int ITEMS, typename Op, typename In>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(In in, int64_t N, Op op, T identity, T *tile_sums)
{
    __shared__ T s_wave[kBlock / kWave];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t wave_base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)w * kWave * ITEMS;
    T acc = identity;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = wave_base + (int64_t)i * kWave + lane;
        if (idx < N) acc = op(acc, in(idx));
    }
    acc = wave_reduce(acc, op);
    if (lane == 0) s_wave[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = identity;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) t = op(t, s_wave[i]);
        tile_sums[blockIdx.x] = t;
    }
}

// exclusive scan of tile sums by one block of 1024 threads, 8 per thread
template <typename T, typename Op>
__global__ __launch_bounds__(1024) void scan_tiles_kernel(T *sums, int64_t ntiles, Op op, T identity,
                                                          T *total_out)
{
    constexpr int kT = 1024, kPer = 8, kW = kT / kWave;
    __shared__ T s_wave[kW];
    __shared__ T s_carry;
    const int t = threadIdx.x, w = t / kWave, lane = lane_id();
    if (t == 0) s_carry = identity;
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += (int64_t)kT * kPer) {
        T v[kPer];
        T loc = identity;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int64_t idx = base + (int64_t)t * kPer + i;
            v[i] = idx < ntiles ? sums[idx] : identity;
            loc = op(loc, v[i]);
        }
        T inc = wave_inclusive(loc, op, identity);
        if (lane == kWave - 1) s_wave[w] = inc;
        __syncthreads();
        T pre = s_carry;
        for (int i = 0; i < w; ++i) pre = op(pre, s_wave[i]);
        // exclusive prefix of this thread's first element
        T excl = shfl_up_t(inc, 1);
        T run = op(pre, lane == 0 ? identity : excl);
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            int64_t idx = base + (int64_t)t * kPer + i;
            if (idx < ntiles) sums[idx] = run;
            run = op(run, v[i]);
        }
        __syncthreads();
        if (t == kT - 1) s_carry = run;
        __syncthreads();
    }
    if (t == 0 && total_out) *total_out = s_carry;
}

template <typename T, int ITEMS, typename Op, typename In, typename Out>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(In in, Out out, int64_t N, Op op, T identity,
                                                            const T *tile_prefix)
{
    __shared__ T s_wave[kBlock / kWave];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int64_t wave_base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)w * kWave * ITEMS;
    T v[ITEMS];
    T acc = identity;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = wave_base + (int64_t)i * kWave + lane;
        v[i] = idx < N ? in(idx) : identity;
        acc = op(acc, v[i]);
    }
    acc = wave_reduce(acc, op);
    if (lane == 0) s_wave[w] = acc;
    __syncthreads();
    T run = tile_prefix[blockIdx.x];
    for (int i = 0; i < w; ++i) run = op(run, s_wave[i]);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        T sc = wave_inclusive(v[i], op, identity);
        int64_t idx = wave_base + (int64_t)i * kWave + lane;
        if (idx < N) out(idx, op(run, sc), v[i]);
        run = op(run, shfl_idx_t(sc, kWave - 1));
    }
}

// Scratch for one scan of N elements.
template <typename T>
struct ScanScratch {
    static size_t bytes_for(int64_t N, int items)
    {
        int64_t tiles = (N + (int64_t)kBlock * items - 1) / ((int64_t)kBlock * items);
        if (tiles < 1) tiles = 1;
        return (size_t)tiles * sizeof(T) + 256;
    }
};

// Launch a scan; `scratch` must hold ScanScratch<T>::bytes_for(N, ITEMS) bytes.
template <typename T, int ITEMS, typename Op, typename In, typename Out>
pm_status scan_launch(In in, Out out, int64_t N, Op op, T identity, void *scratch, hipStream_t s)
{
    if (N <= 0) return PM_OK;
    const int64_t tiles = (N + (int64_t)kBlock * ITEMS - 1) / ((int64_t)kBlock * ITEMS);
    T *sums = (T *)scratch;
    hipLaunchKernelGGL((scan_reduce_kernel<T, ITEMS, Op, In>), dim3((unsigned)tiles), dim3(kBlock), 0, s, in, N, op,
                       identity, sums);
    PM_HIP(hipGetLastError());
    hipLaunchKernelGGL((scan_tiles_kernel<T, Op>), dim3(1), dim3(1024), 0, s, sums, tiles, op, identity,
                       (T *)nullptr);
    PM_HIP(hipGetLastError());
    hipLaunchKernelGGL((scan_apply_kernel<T, ITEMS, Op, In, Out>), dim3((unsigned)tiles), dim3(kBlock), 0, s, in,
                       out, N, op, identity, (const T *)sums);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
