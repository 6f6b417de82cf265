// Enumeration kernels for batches mixing k = 1..12.
#include "enum_dense.hpp"

BDEG_ENUM_INSTANCES(1, 12)
