// Lifetime of library-owned device objects and host-to-device staging
// (internal to libgw).
//
// * Retirement.  An object that enqueued work may still read (a plan's
//   tables, a captured graph and its buffers) is not freed when the library
//   drops it: its destroy function is kept with a HIP event recorded after its
//   last use and runs once that event has completed.  Completion is polled
//   without waiting at the start of later API calls; gw_release waits.
// * Staging.  Host tables reach the device through library-owned pinned
//   buffers: the host data is copied into a buffer whose previous copy has
//   completed (polled, never waited for; the pool grows when every buffer is
//   still in flight) and an asynchronous copy is enqueued on the stream.
// * No-allocation mode.  While a NoAllocScope is alive on a thread, every
//   path that would allocate device memory or create a stream fails with
//   GW_EINVAL instead (used by the fixed-scratch entry point).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

namespace gw {

void retire(int device, hipEvent_t last_use, std::function<void()> destroy);
void sweep_retired();   // runs the destroy functions whose events have completed
void drain_retired();   // waits for every retired object and destroys it

void stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s);
void release_staging();

bool noalloc_mode();
void require_alloc(const char* what);  // throws GW_EINVAL in no-allocation mode

struct NoAllocScope {
    NoAllocScope();
    ~NoAllocScope();
    NoAllocScope(const NoAllocScope&) = delete;
    NoAllocScope& operator=(const NoAllocScope&) = delete;
};

// True when `s` is capturing into a HIP graph (events recorded there would
// become graph nodes).
bool stream_capturing(hipStream_t s);

}  // namespace gw
