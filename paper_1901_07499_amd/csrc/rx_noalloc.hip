// rx_noalloc.hip -- rx_process_frame_noalloc: the receive path with the
// channel estimate in a library-owned device array instead of caller memory,
// for callers that cannot allocate (see include/rx.h).
//
// `scratch` is a file-scope device array; each GPU the library runs on holds
// its own copy at its own address.  Host code never uses the array's name as
// a device address: the address is looked up with hipGetSymbolAddress once
// per device (with that device current) and kept in dev_scratch[].
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "../../include/rx.h"
#include "rx_launch.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) float2 scratch[RX_NOALLOC_SCRATCH_BYTES / sizeof(float2)];

std::atomic<void*> dev_scratch[kMaxDevices];

// This device's copy of `scratch` (nullptr on error).  Concurrent first
// calls on one device look up and store the same address.
float2* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  void* p = dev_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    dev_scratch[dev].store(p, std::memory_order_release);
  }
  return static_cast<float2*>(p);
}

}  // namespace

extern "C" int rx_process_frame_noalloc(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* xhat,
                                        uint8_t* bits, void* hip_stream) {
  // the lookup only reads the array's address; process_frame_in checks every
  // argument before it launches anything, and reports a failed lookup only
  // for a call that would use the buffer
  float2* buf = (plan && n_slots > 0) ? scratch_ptr() : nullptr;
  return rx::process_frame_in(plan, iq, n_slots, xhat, bits, buf, RX_NOALLOC_SCRATCH_BYTES, hip_stream);
}
