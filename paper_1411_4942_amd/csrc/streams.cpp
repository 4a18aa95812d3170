// Side streams (see streams.hpp).
#include "streams.hpp"

#include <array>
#include <map>
#include <mutex>

namespace pm {

hipError_t side_streams(hipStream_t out[2])
{
    static std::mutex mu;
    static std::map<int, std::array<hipStream_t, 2>> made;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = made.find(dev);
    if (it == made.end()) {
        std::array<hipStream_t, 2> ss{};
        for (auto &x : ss)
            if ((e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking)) != hipSuccess) return e;
        it = made.emplace(dev, ss).first;
    }
    out[0] = it->second[0];
    out[1] = it->second[1];
    return hipSuccess;
}

}  // namespace pm
