// HIP-event timing of library launches: a measurement aid for harnesses
// (roofline fractions need the duration of one kernel on the stream it runs on).
#include "prof.hpp"

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace gw {

namespace {

struct Rec {
    hipEvent_t a, b;
};

struct Registry {
    std::mutex mu;
    std::map<std::string, std::vector<Rec>> recs;
    std::vector<hipEvent_t> free_events;
};

std::atomic<bool> g_on{false};

Registry& reg() {
    static Registry* r = new Registry();
    return *r;
}

hipEvent_t take_event(Registry& r) {
    if (!r.free_events.empty()) {
        hipEvent_t e = r.free_events.back();
        r.free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    GW_HIP_TRY(hipEventCreate(&e));
    return e;
}

}  // namespace

bool prof_on() { return g_on.load(std::memory_order_relaxed); }

void prof_enable(bool on) { g_on.store(on); }

void prof_reset() {
    Registry& r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    for (auto& kv : r.recs)
        for (auto& x : kv.second) {
            (void)hipEventSynchronize(x.b);
            r.free_events.push_back(x.a);
            r.free_events.push_back(x.b);
        }
    r.recs.clear();
}

void prof_read(const char* name, int64_t* launches, double* total_ms) {
    Registry& r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    int64_t n = 0;
    double t = 0.0;
    auto it = r.recs.find(name);
    if (it != r.recs.end()) {
        for (auto& x : it->second) {
            GW_HIP_TRY(hipEventSynchronize(x.b));
            float ms = 0.f;
            GW_HIP_TRY(hipEventElapsedTime(&ms, x.a, x.b));
            t += ms;
            ++n;
        }
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = t;
}

ProfScope::ProfScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    if (!prof_on()) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    Registry& r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    a_ = take_event(r);
    GW_HIP_TRY(hipEventRecord(a_, s_));
}

ProfScope::~ProfScope() {
    if (!a_) return;
    Registry& r = reg();
    std::lock_guard<std::mutex> lk(r.mu);
    hipEvent_t b = nullptr;
    try {
        b = take_event(r);
    } catch (...) {
        return;
    }
    if (hipEventRecord(b, s_) != hipSuccess) return;
    r.recs[name_].push_back({a_, b});
}

}  // namespace gw
