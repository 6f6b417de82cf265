// Enumeration kernels for k = 8 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(8, 8)
