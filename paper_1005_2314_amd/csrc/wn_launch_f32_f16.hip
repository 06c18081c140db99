// Launchers of binary32 pools with binary16 output:
// instances of the templates in wn_launch.hpp.

#include "wn_launch.hpp"

WN_LAUNCH_UNIT(float, f32, Half, f16)
