// Enumeration kernels for k = 4 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(4, 4)
