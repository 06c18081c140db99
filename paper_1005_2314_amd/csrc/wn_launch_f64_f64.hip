// Launchers of binary64 pools with binary64 output, and the seeding of binary64 pools:
// instances of the templates in wn_launch.hpp.

#include "wn_launch.hpp"

WN_LAUNCH_UNIT(double, f64, double, f64)

namespace wn {
hipError_t seed_f64(const SeedArgs &a, hipStream_t s) { return seed_n<double>(a, s); }
}  // namespace wn
