// The library's one statically allocated device buffer: the per-request
// statistics partials of wn_fill_stats_noalloc (include/wn.h), the variant of
// wn_fill_stats for callers that cannot allocate device memory.
//
// `scratch` holds kNoAllocRequests partials of 96 bytes (6 MiB).  Every device
// the library's code object is loaded on holds its own copy until the process
// ends, at its own address.  In host code the array's name is only a host-side
// stand-in: its device address comes from hipGetSymbolAddress, called once per
// device with that device current (wn_create does it), and only that address
// is ever passed to a kernel.  All calls on one device share the array; calls
// that overlap on one device race.

#include <mutex>

#include "wn_internal.hpp"

namespace wn {
namespace {

constexpr uint32_t kScratchWords = kNoAllocRequests * uint32_t(sizeof(StatsPartial) / 8);
static_assert(sizeof(StatsPartial) % 8 == 0, "partials are whole words");

static __device__ __align__(256) uint64_t scratch[kScratchWords];

std::mutex g_lock;
StatsPartial *g_addr[kMaxDevices] = {};  // device address of scratch, per device

}  // namespace

hipError_t noalloc_partials(int device, StatsPartial **out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> hold(g_lock);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = static_cast<StatsPartial *>(p);
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace wn
