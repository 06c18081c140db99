// Stand-ins for the device launchers of the library, for a host-only build of
// the C ABI under the host sanitizers (test_host_sanitizers.py).  Every call
// that reaches them needs a device, and the sanitized driver runs where there
// is none, so each returns hipErrorNoDevice.
#include "wn_internal.hpp"

namespace wn {
hipError_t noalloc_partials(int, StatsPartial **out) {
  *out = nullptr;
  return hipErrorNoDevice;
}
hipError_t stats_zero(StatsOut *, hipStream_t) { return hipErrorNoDevice; }
hipError_t zero_words(void *, uint32_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t stats_reduce(const StatsPartial *, uint32_t, StatsOut *, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t seed_f32(const SeedArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t seed_f64(const SeedArgs &, hipStream_t) { return hipErrorNoDevice; }
#define WN_STUB_LAUNCH_UNIT(P, Q)                                                            \
  hipError_t fill_##P##_##Q(const FillArgs &, hipStream_t) { return hipErrorNoDevice; }     \
  hipError_t persistent_##P##_##Q(const FillArgs &, uint32_t, uint32_t, hipStream_t) {      \
    return hipErrorNoDevice;                                                                  \
  }
WN_STUB_LAUNCH_UNIT(f32, f32)
WN_STUB_LAUNCH_UNIT(f32, bf16)
WN_STUB_LAUNCH_UNIT(f32, f16)
WN_STUB_LAUNCH_UNIT(f64, f64)
WN_STUB_LAUNCH_UNIT(f64, f32)
WN_STUB_LAUNCH_UNIT(f64, bf16)
WN_STUB_LAUNCH_UNIT(f64, f16)
}  // namespace wn
