// Device memory for the library: a caching allocator.
//
// A freed block goes to a per-device free list with the stream that freed it
// and an event recorded there (one event for a whole batch of frees).  A
// later allocation of a similar size takes the block.  On the same stream
// the stream order already puts every new use after the old ones, so no wait
// is queued.  On another stream the new stream waits for the event (a
// device-side wait), so reuse across streams stays ordered.  Each event
// record or wait is a packet the GPU processes between kernels, which is why
// both are kept to what ordering needs.  New blocks come from hipMalloc;
// when that runs out of memory the free lists are released and the
// allocation retried.  pm_release_cached_memory() returns every cached block.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/pathsamp.h"

namespace pm {

void set_error(const std::string &msg);

namespace {

// an event shared by the blocks of one batch of frees, destroyed with the last
struct SharedEvent {
    hipEvent_t ev = nullptr;
    ~SharedEvent()
    {
        if (ev) (void)hipEventDestroy(ev);
    }
};

struct FreeBlock {
    void *ptr;
    size_t bytes;
    hipStream_t stream;                 // the freeing stream
    std::shared_ptr<SharedEvent> ready; // recorded on it (null: already idle)
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
        if (kv.second.ready) (void)hipEventSynchronize(kv.second.ready->ev);
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
        if (b.ready && b.stream != s) {
            e = hipStreamWaitEvent(s, b.ready->ev, 0);
            if (e != hipSuccess) {
                (void)hipEventSynchronize(b.ready->ev);
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

void dev_free_batch(void *const *ps, size_t count, hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    std::shared_ptr<SharedEvent> ready;  // one event for the batch, made at its first block of ours
    bool waited = false;
    for (size_t i = 0; i < count; ++i) {
        void *p = ps[i];
        if (!p) continue;
        auto it = c.live.find(p);
        if (it == c.live.end()) continue;  // not ours (or freed on another device)
        if (!ready && !waited) {
            auto ev = std::make_shared<SharedEvent>();
            if (hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming) == hipSuccess &&
                hipEventRecord(ev->ev, s) == hipSuccess) {
                ready = ev;
            } else {
                // cannot mark the point of release: wait for the stream instead
                (void)hipStreamSynchronize(s);
                waited = true;
            }
        }
        FreeBlock b{p, it->second, s, ready};
        c.live.erase(it);
        c.free_blocks.emplace(b.bytes, b);
        c.cached_bytes += b.bytes;
    }
}

void dev_free(void *p, hipStream_t s) { dev_free_batch(&p, 1, s); }

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
