// Launchers of binary64 pools with binary32 output:
// instances of the templates in wn_launch.hpp.

#include "wn_launch.hpp"

WN_LAUNCH_UNIT(double, f64, float, f32)
