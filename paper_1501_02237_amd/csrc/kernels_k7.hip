// Enumeration kernels for k = 7 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(7, 7)
