// Enumeration kernels for k = 14: both lane-group variants, plain, counting and
// cell-listing modes (instantiated from enum_device.hpp).
#include "enum_dense.hpp"
BDEG_ENUM_INSTANCES(14, 14)
