// Enumeration kernels for batches mixing k = 1..7.
#include "enum_dense.hpp"

BDEG_ENUM_INSTANCES(1, 7)
