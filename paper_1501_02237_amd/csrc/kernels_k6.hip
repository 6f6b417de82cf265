// Enumeration kernels for k = 6 (all lane-group counts, timed and counting variants).
#include "enum_device.hpp"

BDEG_ENUM_INSTANCES(6, 6)
