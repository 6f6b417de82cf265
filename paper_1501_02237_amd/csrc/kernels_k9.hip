// Enumeration kernels for k = 9 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(9, 9)
