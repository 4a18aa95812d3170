// Side streams for work that can run beside the caller's stream on the
// same device (fork-join through events).
#pragma once

#include <hip/hip_runtime.h>

namespace pm {

// Two streams per device (default priority, non-blocking), created on first
// use on the current device and kept for the life of the process.  The row
// build runs its classes of long rows on them beside the others.
hipError_t side_streams(hipStream_t out[2]);

// Fork-join on side streams: on construction the side streams wait for
// everything enqueued on s so far; join() makes s wait for everything
// enqueued on them since (waiting on the host for a stream whose event calls
// fail), and the destructor joins if that has not happened.
struct Fork {
    hipStream_t s;
    hipStream_t *side;
    int k;
    bool joined = false;
    hipError_t status = hipSuccess;

    Fork(hipStream_t s_, hipStream_t *side_, int k_) : s(s_), side(side_), k(k_)
    {
        hipEvent_t e = nullptr;
        status = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (status == hipSuccess) status = hipEventRecord(e, s);
        for (int i = 0; i < k && status == hipSuccess; ++i) status = hipStreamWaitEvent(side[i], e, 0);
        if (e) (void)hipEventDestroy(e);
        if (status != hipSuccess) joined = true;  // the caller returns before launching anything
    }
    hipError_t join()
    {
        if (joined) return hipSuccess;
        joined = true;
        hipError_t r = hipSuccess;
        for (int i = 0; i < k; ++i) {
            hipEvent_t e = nullptr;
            hipError_t x = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (x == hipSuccess) x = hipEventRecord(e, side[i]);
            if (x == hipSuccess) x = hipStreamWaitEvent(s, e, 0);
            if (e) (void)hipEventDestroy(e);
            if (x != hipSuccess) {
                (void)hipStreamSynchronize(side[i]);
                r = x;
            }
        }
        return r;
    }
    ~Fork() { (void)join(); }
    Fork(const Fork &) = delete;
    Fork &operator=(const Fork &) = delete;
};

}  // namespace pm
