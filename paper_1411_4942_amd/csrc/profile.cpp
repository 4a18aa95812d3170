// Per-kernel HIP event timing (see profile.hpp).
#include "profile.hpp"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/pathsamp.h"

namespace pm {

void set_error(const std::string &msg);

namespace {

struct Pending {
    std::string name;
    hipEvent_t a, b;
};

struct Totals {
    uint64_t launches = 0;
    double ms = 0.0;
};

std::atomic<bool> g_on{false};
std::atomic<bool> g_all{true};  // no selection: every scope is recorded
std::mutex g_mu;
std::set<std::string> g_selected;
std::vector<Pending> g_pending;
std::map<std::string, Totals> g_totals;

void resolve_locked()
{
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            Totals &t = g_totals[p.name];
            t.launches += 1;
            t.ms += ms;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}

}  // namespace

bool profiling() { return g_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s)
{
    if (!profiling()) return;
    if (!g_all.load(std::memory_order_relaxed)) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_selected.count(name_)) return;
    }
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        a_ = b_ = nullptr;
        return;
    }
    (void)hipEventRecord(a_, s_);
}

ProfScope::~ProfScope()
{
    if (!a_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(Pending{name_, a_, b_});
}

}  // namespace pm

extern "C" {

pm_status pm_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(pm::g_mu);
    pm::resolve_locked();
    pm::g_totals.clear();
    pm::g_on.store(on != 0);
    return PM_OK;
}

pm_status pm_profile_select(const char *names)
{
    std::lock_guard<std::mutex> lk(pm::g_mu);
    pm::g_selected.clear();
    const std::string all = names ? names : "";
    size_t a = 0;
    while (a <= all.size()) {
        size_t b = all.find(',', a);
        if (b == std::string::npos) b = all.size();
        if (b > a) pm::g_selected.insert(all.substr(a, b - a));
        a = b + 1;
    }
    pm::g_all.store(pm::g_selected.empty());
    return PM_OK;
}

pm_status pm_profile_read(pm_profile_entry *out, int32_t capacity, int32_t *count)
{
    if (!count || capacity < 0 || (capacity > 0 && !out)) {
        pm::set_error("pm_profile_read: bad arguments");
        return PM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(pm::g_mu);
    pm::resolve_locked();
    int32_t i = 0;
    for (auto &kv : pm::g_totals) {
        if (i < capacity) {
            std::memset(&out[i], 0, sizeof(out[i]));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.launches;
            out[i].total_ms = kv.second.ms;
        }
        ++i;
    }
    *count = i;
    return PM_OK;
}

}  // extern "C"
