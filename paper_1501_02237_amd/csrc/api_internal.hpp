// Shared between the C-ABI front end and the serving engine.
#pragma once

#include <vector>

#include "runtime.hpp"

namespace bdeg {

// Host prologue of one system; true when device work is needed (then `hs`
// is filled and res.status == BDEG_PENDING).
bool prepare_one(const int64_t *A, int m, int n, uint64_t seed, int lift_bits, int index, bdeg_result &res,
                 HostSys &hs);
int prepare_many(const int64_t *A_concat, const int32_t *m, const int32_t *n, int count, uint64_t seed,
                 int lift_bits, std::vector<bdeg_result> &res, std::vector<HostSys> &dev);
int finish_device(Device *D, std::vector<HostSys> &dev, std::vector<bdeg_result> &res, Job *first,
                  DevCounters *cnt_out);

} // namespace bdeg
