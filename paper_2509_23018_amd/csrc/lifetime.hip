// Deferred release, pinned staging and the no-allocation mode (lifetime.hpp).
#include "lifetime.hpp"

#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace gw {
namespace {

struct Retired {
    int device;
    hipEvent_t ev;
    std::function<void()> destroy;
};

struct RetireList {
    std::mutex mu;
    std::vector<Retired> items;
};

RetireList& retired() {
    static RetireList* r = new RetireList();  // leaked on purpose: no teardown order issues
    return *r;
}

struct Staging {
    int device;
    void* host;
    size_t bytes;
    hipEvent_t ev;  // recorded after the copy that last read the buffer
};

struct StagingPool {
    std::mutex mu;
    std::vector<Staging> bufs;
};

StagingPool& staging() {
    static StagingPool* p = new StagingPool();
    return *p;
}

thread_local int t_noalloc = 0;

}  // namespace

void retire(int device, hipEvent_t last_use, std::function<void()> destroy) {
    RetireList& r = retired();
    std::lock_guard<std::mutex> lk(r.mu);
    r.items.push_back(Retired{device, last_use, std::move(destroy)});
}

void sweep_retired() {
    std::vector<Retired> done;
    {
        RetireList& r = retired();
        std::lock_guard<std::mutex> lk(r.mu);
        if (r.items.empty()) return;
        int cur = 0;
        (void)hipGetDevice(&cur);
        std::vector<Retired> keep;
        for (auto& it : r.items) {
            // hipEventQuery needs the event's device to be current
            if (it.device != cur) (void)hipSetDevice(it.device);
            const hipError_t q = it.ev ? hipEventQuery(it.ev) : hipSuccess;
            if (it.device != cur) (void)hipSetDevice(cur);
            if (q == hipErrorNotReady) {
                keep.push_back(std::move(it));
            } else {
                (void)hipGetLastError();
                done.push_back(std::move(it));
            }
        }
        r.items.swap(keep);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& it : done) {
        (void)hipSetDevice(it.device);
        it.destroy();
    }
    (void)hipSetDevice(cur);
}

void drain_retired() {
    std::vector<Retired> all;
    {
        RetireList& r = retired();
        std::lock_guard<std::mutex> lk(r.mu);
        all.swap(r.items);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& it : all) {
        (void)hipSetDevice(it.device);
        if (it.ev) (void)hipEventSynchronize(it.ev);
        it.destroy();
    }
    (void)hipSetDevice(cur);
}

void stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    int dev = 0;
    GW_HIP_TRY(hipGetDevice(&dev));
    StagingPool& p = staging();
    std::lock_guard<std::mutex> lk(p.mu);
    Staging* use = nullptr;
    for (auto& b : p.bufs) {
        if (b.device != dev || b.bytes < bytes) continue;
        const hipError_t q = hipEventQuery(b.ev);
        if (q == hipErrorNotReady) continue;
        (void)hipGetLastError();
        if (!use || b.bytes < use->bytes) use = &b;
    }
    if (!use) {
        require_alloc("pinned staging buffer");
        Staging b{dev, nullptr, std::max<size_t>(bytes, size_t(1) << 16), nullptr};
        GW_HIP_TRY(hipHostMalloc(&b.host, b.bytes, hipHostMallocDefault));
        const hipError_t e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(b.host);
            GW_HIP_TRY(e);
        }
        p.bufs.push_back(b);
        use = &p.bufs.back();
    }
    std::memcpy(use->host, src, bytes);
    GW_HIP_TRY(hipMemcpyAsync(dst, use->host, bytes, hipMemcpyHostToDevice, s));
    GW_HIP_TRY(hipEventRecord(use->ev, s));
}

void release_staging() {
    StagingPool& p = staging();
    std::lock_guard<std::mutex> lk(p.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& b : p.bufs) {
        (void)hipSetDevice(b.device);
        (void)hipEventSynchronize(b.ev);
        (void)hipEventDestroy(b.ev);
        (void)hipHostFree(b.host);
    }
    p.bufs.clear();
    (void)hipSetDevice(cur);
}

bool noalloc_mode() { return t_noalloc > 0; }

void require_alloc(const char* what) {
    if (t_noalloc > 0)
        throw Error{-1, std::string("this call allocates nothing, but it would need a new ") + what +
                            " (make one ordinary call with the same grid, G list and options "
                            "first)"};
}

NoAllocScope::NoAllocScope() { ++t_noalloc; }
NoAllocScope::~NoAllocScope() { --t_noalloc; }

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st != hipStreamCaptureStatusNone;
}

}  // namespace gw
