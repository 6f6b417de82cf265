// Host runtime: device context, device-resident jobs, graph replay, tie retry.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "bdeg_internal.hpp"

namespace bdeg {

struct Device {
  int dev = -1;
  hipStream_t stream = nullptr;
  int cus = 0;
  std::mutex mu; // serialises use of `stream` and the shared scratch job
};
// Process-wide device context; status receives BDEG_OK or BDEG_E_DEVICE.
Device *device_get(int *status);
int device_select(int dev);

// Host side of one device system (k >= 1, certified bounds).
struct HostSys {
  int input_index;   // index in the caller's batch
  int N, k, lift_bits;
  uint32_t attempt;
  uint64_t seed;
  std::vector<int32_t> pts; // N x k
};

// Device buffers for a set of systems and their tiles.
struct Job {
  std::vector<SysDesc> sys;
  std::vector<int32_t> pts;
  std::vector<Tile> tiles;
  int kmin = 0, kmax = 0;
  bool explicit_heights = false;
  std::vector<int64_t> heights; // when explicit

  SysDesc *d_sys = nullptr;
  int32_t *d_pts = nullptr;
  int64_t *d_hts = nullptr;
  Tile *d_tiles = nullptr;
  SysAcc *d_acc = nullptr;
  DevCounters *d_cnt = nullptr; // (1 + RETIE_ROUNDS) * MAX_RANGES blocks: one per launch range and round
  uint32_t *d_rerun = nullptr;  // RETIE_ROUNDS blocks of (systems + 1) redraw flags
  size_t cap_sys = 0, cap_pts = 0, cap_hts = 0, cap_tiles = 0, cap_acc = 0, cap_rerun = 0;

  // units are ordered by launch range: lane-group variant and k class (the
  // mixed-k kernels cover k <= MIXED_K_MAX, deeper systems get single-k
  // kernels); one launch, with its own counter block, per range present
  struct VariantRange {
    bool single;
    bool dense; // the lane-dense kernel (SYS_DENSE systems)
    int kclass; // 0: mixed-k kernel; else the single k
    int klo, khi;
    uint32_t start, count;
  };
  std::vector<VariantRange> granges;

  LaunchShape shape;
  ~Job();
  void release();
};

// Work schedule of a batch, per bucket of systems with the same k and the same
// smallest lane-group width (npad_log2_for(N)): the kernel (lane-dense, for
// systems it is certified for, or lanes as points), the lane-group width the
// lanes-as-points kernel runs with (npad_log2 >= the smallest; 6 = one group
// per wavefront, the single-group kernel variant) and the work-unit size cap.  Chosen by the
// autotuner (tune.cpp) and persisted as a JSON table.
struct BucketSchedule {
  int dense = -1;         // kernel: 1 lane-dense, 0 lanes as points, -1 unset (lane-dense when certified)
  int npad_log2 = 0;      // 0: unset (the default: the smallest width)
  uint64_t unit_cost = 0; // 0: unset (the default: choose_max_cost of the whole job)
  float ms = 0;           // measured device time of the bucket's tuning set with this schedule
  int systems = 0;        // systems in the tuning set
};
struct ScheduleTable {
  BucketSchedule e[BDEG_MAX_K + 1][7]; // [k][smallest npad_log2]
  bool any = false;
};
// The table bdeg_batch_create uses: read once per process from the file named
// by BDEG_TUNE_TABLE, else tuning/gfx950.json beside the library; empty when
// neither exists.
const ScheduleTable &schedule_table();
int schedule_read(const char *path, ScheduleTable &t);
int schedule_write(const char *path, const ScheduleTable &t);

// Build device descriptors and tiles for `systems` (seeded lifting) into job;
// with `sched`, systems of a bucket it sets use that bucket's schedule.
void job_build_seeded(Job &job, const std::vector<HostSys> &systems, uint64_t max_cost,
                      const ScheduleTable *sched = nullptr);
// Order units by (kernel variant, decreasing cost) and record the variant ranges.
void job_order_units(Job &job, std::vector<TileC> &tc);
// index of a kernel variant among the per-(k, variant) counter blocks of the serving engine
inline int group_slot(bool single, bool dense) { return dense ? 2 : single ? 1 : 0; }
constexpr int GROUP_SLOTS = 3;
// Enumeration schedule of the process (bdeg_set_schedule): BDEG_SCHED_AUTO
// runs certified systems with k >= 3 in the lane-dense kernel.
int schedule_mode();
int schedule_set(int schedule);
// deepest k of the mixed-k kernels; launch ranges of a job (each has a counter block)
constexpr int MIXED_K_MAX = 12;
constexpr int MAX_RANGES = 3 * (1 + BDEG_MAX_K - MIXED_K_MAX);
// redraw rounds inside one replayable device pass (a prepared batch): after
// the first enumeration, each round redraws the liftings of the tied systems
// and enumerates their units again; ties left after the last round are
// redrawn by the host
constexpr int RETIE_ROUNDS = 3;
constexpr int CNT_BLOCKS = (1 + RETIE_ROUNDS) * MAX_RANGES;
// Upload (growing buffers as needed).
int job_upload(Job &job);
// Enqueue clear + lift (pre) and the enumeration; job_launch does both.
int job_launch_pre(Job &job, hipStream_t stream);
int job_launch_enum(Job &job, hipStream_t stream, int round = 0);
// Replayable seeded pass: reset every system to attempt 0 and lift (instead of
// job_launch_pre), and the in-pass redraw round r = 1..RETIE_ROUNDS (retie
// kernel, then job_launch_enum(job, stream, r)).
int job_launch_reset(Job &job, hipStream_t stream);
int job_launch_retie(Job &job, hipStream_t stream, int round);
int job_launch(Job &job, hipStream_t stream, hipEvent_t ev_kernel_start = nullptr,
               hipEvent_t ev_kernel_end = nullptr);
// Copy accumulators back (synchronous on stream).
int job_collect(Job &job, hipStream_t stream, std::vector<SysAcc> &acc, DevCounters *cnt);

// Work-unit size cap: about 16 units per resident wavefront, never below
// `floor` candidates.  Throughput work uses the default floor (fewer, longer
// units: less prefix re-derivation per candidate); latency work (a lone small
// request) passes a smaller one to spread over more wavefronts.
constexpr uint64_t UNIT_FLOOR = 512;
// Largest work unit: a unit's step budget, (k + 3) steps per candidate with
// k <= 18, must fit the device's signed 32-bit budget count.
constexpr uint64_t MAX_UNIT_CANDIDATES = 1ull << 26;
uint64_t choose_max_cost(uint64_t total_candidates, int waves, uint64_t floor = UNIT_FLOOR);
int default_waves(int kmin, int kmax, int waves_per_block);

} // namespace bdeg
