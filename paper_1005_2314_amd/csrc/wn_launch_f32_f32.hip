// Launchers of binary32 pools with binary32 output, and the seeding of binary32 pools:
// instances of the templates in wn_launch.hpp.

#include "wn_launch.hpp"

WN_LAUNCH_UNIT(float, f32, float, f32)

namespace wn {
hipError_t seed_f32(const SeedArgs &a, hipStream_t s) { return seed_n<float>(a, s); }
}  // namespace wn
