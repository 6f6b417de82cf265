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
// Arguments of the point-set entry points: shape, |h| < 2^40, device bound.
int check_points(const int32_t *points, const int64_t *heights, int N, int k);
// One caller point set with explicit heights, candidates of colex rank in
// [rank_lo, rank_hi), work units of at most max_cost candidates (0: the
// default size for the current device).
void points_job(Job &job, const int32_t *points, const int64_t *heights, int N, int k, uint64_t rank_lo,
                uint64_t rank_hi, uint64_t max_cost = 0);
// Collect `first` (an already-launched job holding all of `dev` in order) or
// launch the systems, then redraw the tied ones on the host until none ties.
// *redraws_out (optional): systems whose lifting was redrawn inside `first`'s
// device pass.
int finish_device(Device *D, std::vector<HostSys> &dev, std::vector<bdeg_result> &res, Job *first,
                  DevCounters *cnt_out, int32_t *redraws_out = nullptr);

} // namespace bdeg
