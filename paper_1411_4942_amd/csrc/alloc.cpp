// Device memory for the library: a caching allocator.
//
// A freed block goes to a per-device free list together with an event
// recorded on the stream that freed it; a later allocation of a similar size
// takes the block and makes its own stream wait for that event (a device-side
// wait), so reuse across streams stays ordered.  New blocks come from
// hipMalloc; when that runs out of memory the free lists are released and the
// allocation retried.  pm_release_cached_memory() returns every cached block.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/pathsamp.h"

namespace pm {

void set_error(const std::string &msg);

namespace {

struct FreeBlock {
    void *ptr;
    size_t bytes;
    hipEvent_t ready;  // recorded on the freeing stream (null: already idle)
};

struct DeviceCache {
    std::multimap<size_t, FreeBlock> free_blocks;  // by size
    std::unordered_map<void *, size_t> live;       // block -> size
    size_t cached_bytes = 0;
};

constexpr int kMaxDevices = 64;
std::mutex g_mu;
DeviceCache g_cache[kMaxDevices];

size_t round_size(size_t bytes)
{
    if (bytes == 0) bytes = 1;
    const size_t big = size_t(2) << 20;
    if (bytes >= big) return (bytes + big - 1) / big * big;  // 2 MiB granules
    size_t r = 256;
    while (r < bytes) r <<= 1;  // powers of two below 2 MiB
    return r;
}

void release_all_locked(int dev)
{
    DeviceCache &c = g_cache[dev];
    for (auto &kv : c.free_blocks) {
        if (kv.second.ready) {
            (void)hipEventSynchronize(kv.second.ready);
            (void)hipEventDestroy(kv.second.ready);
        }
        (void)hipFree(kv.second.ptr);
    }
    c.free_blocks.clear();
    c.cached_bytes = 0;
}

}  // namespace

pm_status dev_alloc(void **p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error(std::string("dev_alloc: hipGetDevice: ") + hipGetErrorString(e));
        return PM_EDEVICE;
    }
    const size_t want = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    // reuse a cached block of the same size class (up to 1/8 larger for big blocks)
    auto it = c.free_blocks.lower_bound(want);
    if (it != c.free_blocks.end() && it->first <= want + want / 8) {
        FreeBlock b = it->second;
        c.free_blocks.erase(it);
        c.cached_bytes -= b.bytes;
        if (b.ready) {
            e = hipStreamWaitEvent(s, b.ready, 0);
            (void)hipEventDestroy(b.ready);
            if (e != hipSuccess) {
                (void)hipFree(b.ptr);
                set_error(std::string("dev_alloc: hipStreamWaitEvent: ") + hipGetErrorString(e));
                return PM_EDEVICE;
            }
        }
        c.live[b.ptr] = b.bytes;
        *p = b.ptr;
        return PM_OK;
    }
    void *q = nullptr;
    e = hipMalloc(&q, want);
    if (e == hipErrorOutOfMemory && !c.free_blocks.empty()) {
        (void)hipGetLastError();
        release_all_locked(dev);
        e = hipMalloc(&q, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("hipMalloc(") + std::to_string(want) + "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PM_ENOMEM : PM_EDEVICE;
    }
    c.live[q] = want;
    *p = q;
    return PM_OK;
}

void dev_free(void *p, hipStream_t s)
{
    if (!p) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not ours (or freed on another device)
    FreeBlock b{p, it->second, nullptr};
    c.live.erase(it);
    if (hipEventCreateWithFlags(&b.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(b.ready, s) != hipSuccess) {
        // cannot mark the point of release: wait for the stream instead
        if (b.ready) (void)hipEventDestroy(b.ready);
        b.ready = nullptr;
        (void)hipStreamSynchronize(s);
    }
    c.free_blocks.emplace(b.bytes, b);
    c.cached_bytes += b.bytes;
}

}  // namespace pm

extern "C" pm_status pm_release_cached_memory(void)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= pm::kMaxDevices) {
        pm::set_error("pm_release_cached_memory: no current device");
        return PM_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(pm::g_mu);
    pm::release_all_locked(dev);
    return PM_OK;
}
