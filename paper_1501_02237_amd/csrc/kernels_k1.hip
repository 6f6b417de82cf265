// Enumeration kernels for k = 1 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(1, 1)
