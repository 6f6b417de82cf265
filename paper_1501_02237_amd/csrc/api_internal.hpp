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
// Collect `first` (an already-launched job holding all of `dev` in order) or
// launch the systems, then redraw the tied ones on the host until none ties.
// *redraws_out (optional): systems whose lifting was redrawn inside `first`'s
// device pass.
int finish_device(Device *D, std::vector<HostSys> &dev, std::vector<bdeg_result> &res, Job *first,
                  DevCounters *cnt_out, int32_t *redraws_out = nullptr);

} // namespace bdeg
