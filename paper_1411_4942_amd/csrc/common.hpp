// Shared device/host helpers of the pathsamp HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/pathsamp.h"

namespace pm {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kBlock = 256;   // threads per block for streaming kernels

// ---------------------------------------------------------------------------
// error plumbing (host)
// ---------------------------------------------------------------------------

void set_error(const std::string &msg);

struct Status {
    pm_status code = PM_OK;
};

#define PM_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::pm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
            return e_ == hipErrorOutOfMemory ? PM_ENOMEM : PM_EDEVICE;                    \
        }                                                                                 \
    } while (0)

#define PM_TRY(expr)                 \
    do {                             \
        pm_status s_ = (expr);       \
        if (s_ != PM_OK) return s_;  \
    } while (0)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of: two
// 32x32->64 products (word 0 by M0, word 2 by M1); the new words are
// (hi(w2 M1) ^ w1 ^ k0, lo(w2 M1), hi(w0 M0) ^ w3 ^ k1, lo(w0 M0)); the key
// advances by the Weyl constants (W0, W1) between rounds.
struct U32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = c.x * M0, hi0 = __umulhi(c.x, M0);
        uint32_t lo1 = c.z * M1, hi1 = __umulhi(c.z, M1);
        c = U32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Exact uniform integer in [0, R) for sample `id` of sampler `tag` (R >= 1):
// 64-bit candidates (w0 | w1 << 32) then (w2 | w3 << 32) of Philox at counter
// (id_lo, id_hi, tag, attempt), attempt = 0, 1, ...; each candidate goes
// through Lemire's multiply-and-reject (ACM TOMACS 2019).
__device__ __forceinline__ uint64_t lemire_try(uint64_t x, uint64_t R, bool &ok)
{
    uint64_t lo = x * R;
    uint64_t hi = __umul64hi(x, R);
    ok = true;
    if (lo < R) {
        uint64_t t = (0ull - R) % R;  // (2^64 - R) mod R; rare path
        ok = lo >= t;
    }
    return hi;
}

__device__ __forceinline__ uint64_t draw_bounded(uint64_t seed, uint32_t tag, uint64_t id, uint64_t R)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t attempt = 0;; ++attempt) {
        U32x4 w = philox4x32_10(U32x4{(uint32_t)id, (uint32_t)(id >> 32), tag, attempt}, k0, k1);
        bool ok;
        uint64_t r = lemire_try((uint64_t)w.x | ((uint64_t)w.y << 32), R, ok);
        if (ok) return r;
        r = lemire_try((uint64_t)w.z | ((uint64_t)w.w << 32), R, ok);
        if (ok) return r;
    }
}

// q = a / d, r = a % d for a < 2^63 and 0 < d < 2^31 with a / d < 2^32:
// a double-precision quotient (relative error 2^-52, so the truncated value is
// off by at most one) corrected with exact integer arithmetic.
__device__ __forceinline__ void divmod_small(uint64_t a, uint32_t d, uint64_t &q, uint64_t &r)
{
    uint64_t qq = (uint64_t)((double)a / (double)d);
    int64_t rr = (int64_t)a - (int64_t)(qq * (uint64_t)d);
    while (rr < 0) {
        qq -= 1;
        rr += d;
    }
    while (rr >= (int64_t)d) {
        qq += 1;
        rr -= d;
    }
    q = qq;
    r = (uint64_t)rr;
}

// wave-wide sums
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// fill kernel (used instead of memset so that capture stays plain kernels)
template <typename T>
__global__ void fill_kernel(T *p, T value, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = value;
}

// Blocks for n items at `threads` per block, capped.  Streaming kernels pass
// a cap that is never reached (a flat grid, one item per thread): on MI355X a
// flat copy measured 6.2 TB/s against 4.6 TB/s for 8192 blocks striding
// over the same array.
inline int grid_for(int64_t n, int threads, int max_blocks = 65536)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

// bits needed for the values 0 .. max_key
inline int bits_for(uint64_t max_key)
{
    int b = 0;
    while (b < 64 && (max_key >> b) != 0) ++b;
    return b;
}

template <typename T>
inline pm_status fill_async(T *p, T value, int64_t n, hipStream_t s)
{
    if (n <= 0) return PM_OK;
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n, kBlock, 1 << 22)), dim3(kBlock), 0, s, p, value, n);
    PM_HIP(hipGetLastError());
    return PM_OK;
}

}  // namespace pm
