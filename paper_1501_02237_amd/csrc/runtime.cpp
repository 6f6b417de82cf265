// Host runtime: one device context per process, device-resident jobs.
#include "runtime.hpp"

#include <stdlib.h>

#include <algorithm>
#include <atomic>

namespace bdeg {

static Device g_device;
static std::atomic<int> g_schedule{BDEG_SCHED_AUTO};

int schedule_mode() { return g_schedule.load(std::memory_order_relaxed); }
int schedule_set(int s) {
  if (s != BDEG_SCHED_AUTO && s != BDEG_SCHED_POINTS) return BDEG_E_ARG;
  g_schedule.store(s, std::memory_order_relaxed);
  return BDEG_OK;
}

bool dense_ok(const int32_t *pts, int N, int k, uint64_t height_span) {
  if (k < 3 || schedule_mode() != BDEG_SCHED_AUTO) return false;
  return device_bounds_ok(pts, N, k, height_span, 30, 59);
}
static std::once_flag g_once;
static int g_status = BDEG_E_DEVICE;
static int g_requested = -1;

int device_select(int dev) {
  if (g_device.dev >= 0) return BDEG_E_STATE;
  g_requested = dev;
  return BDEG_OK;
}

Device *device_get(int *status) {
  std::call_once(g_once, [] {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return;
    int dev = 0;
    if (g_requested >= 0) {
      if (g_requested >= count) return;
      dev = g_requested;
    } else {
      const char *env = getenv("BDEG_DEVICE");
      if (env) dev = atoi(env);
      else if (hipGetDevice(&dev) != hipSuccess) dev = 0;
      if (dev < 0 || dev >= count) return;
    }
    if (hipSetDevice(dev) != hipSuccess) return;
    if (hipStreamCreateWithFlags(&g_device.stream, hipStreamNonBlocking) != hipSuccess) return;
    g_device.dev = dev;
    g_device.cus = device_cu_count();
    g_status = BDEG_OK;
  });
  if (status) *status = g_status;
  if (g_status != BDEG_OK) return nullptr;
  (void)hipSetDevice(g_device.dev);
  return &g_device;
}

int default_waves(int kmin, int kmax, int waves_per_block) {
  if (kmin != kmax && kmax > MIXED_K_MAX) kmin = kmax; // the deepest launch sets the grid
  int blocks = max_enum_blocks(kmin, kmax, waves_per_block, false);
  return blocks > 0 ? blocks * waves_per_block : 1024;
}

// Subtree size cap (a unit re-derives its prefix, which costs a few levels).
// At most 2^26 candidates per unit, so that a unit's step budget, (k + 3)
// steps per candidate with k <= 18, stays below the device's signed 32-bit
// budget count however large the job.
uint64_t choose_max_cost(uint64_t total, int waves, uint64_t floor) {
  uint64_t per = total / ((uint64_t)(waves > 0 ? waves : 1) * 16);
  if (per > MAX_UNIT_CANDIDATES) per = MAX_UNIT_CANDIDATES;
  return per < floor ? floor : per;
}


void job_build_seeded(Job &job, const std::vector<HostSys> &systems, uint64_t max_cost,
                      const ScheduleTable *sched) {
  job.sys.clear();
  job.pts.clear();
  job.tiles.clear();
  job.kmin = 1 << 30;
  job.kmax = 0;
  job.explicit_heights = false;
  int ht = 0;
  std::vector<TileC> tc;
  for (size_t s = 0; s < systems.size(); s++) {
    const HostSys &h = systems[s];
    SysDesc d;
    d.N = h.N;
    d.k = h.k;
    d.pt_off = (int32_t)job.pts.size();
    d.ht_off = ht;
    d.lift_bits = h.lift_bits;
    d.npad_log2 = npad_log2_for(h.N);
    uint64_t cost = max_cost;
    bool dense = dense_ok(h.pts.data(), h.N, h.k, (1ull << h.lift_bits) - 1);
    if (sched) {
      const BucketSchedule &b = sched->e[h.k][d.npad_log2];
      if (b.npad_log2 >= d.npad_log2 && b.npad_log2 <= 6) d.npad_log2 = b.npad_log2;
      if (b.unit_cost > 0) cost = b.unit_cost;
      if (b.dense == 0) dense = false;
    }
    // every system draws from the single-system stream (index 0), so its
    // liftings, and hence attempts and cells, do not depend on its position
    // in a batch: a batched result equals the one-shot result exactly
    d.lift_key = lift_key(h.seed, 0u, h.attempt);
    d.seed = h.seed;
    d.sys_index = 0;
    d.flags = dense ? SYS_DENSE | SYS_SORTED : 0; // every unit of the system
    job.sys.push_back(d);
    job.pts.insert(job.pts.end(), h.pts.begin(), h.pts.end());
    ht += h.N;
    job.kmax = std::max(job.kmax, h.k);
    job.kmin = std::min(job.kmin, h.k);
    tiles_full(h.N, h.k, (uint32_t)s, cost, tc);
  }
  if (job.kmin > job.kmax) job.kmin = job.kmax;
  job_order_units(job, tc);
  job.heights.assign(ht, 0);
}

void job_order_units(Job &job, std::vector<TileC> &tc) {
  // k class: 0 for the mixed-k kernels, k itself above them
  auto kclass = [&](const TileC &t) {
    const int k = job.sys[t.t.sys].k;
    return (job.kmin != job.kmax && k <= MIXED_K_MAX) ? 0 : k;
  };
  // kernel variant: 0 lane groups, 1 one point group per wavefront, 2 lane-dense
  auto variant = [&](const TileC &t) {
    const SysDesc &d = job.sys[t.t.sys];
    return (d.flags & SYS_DENSE) ? 2 : d.npad_log2 == 6 ? 1 : 0;
  };
  std::stable_sort(tc.begin(), tc.end(), [&](const TileC &a, const TileC &b) {
    const int ga = variant(a), gb = variant(b);
    if (ga != gb) return ga < gb;
    const int ka = kclass(a), kb = kclass(b);
    if (ka != kb) return ka < kb;
    return a.cost > b.cost;
  });
  job.tiles.resize(tc.size());
  job.granges.clear();
  for (size_t i = 0; i < tc.size(); i++) {
    job.tiles[i] = tc[i].t;
    const int v = variant(tc[i]);
    const bool g = v == 1, dn = v == 2;
    const int kc = kclass(tc[i]);
    if (job.granges.empty() || job.granges.back().single != g || job.granges.back().dense != dn ||
        job.granges.back().kclass != kc) {
      Job::VariantRange r;
      r.single = g;
      r.dense = dn;
      r.kclass = kc;
      r.klo = kc != 0 ? kc : job.kmin;
      r.khi = kc != 0 ? kc : std::min(job.kmax, MIXED_K_MAX);
      r.start = (uint32_t)i;
      r.count = 0;
      job.granges.push_back(r);
    }
    job.granges.back().count++;
  }
}

template <typename T>
static int grow(T **ptr, size_t *cap, size_t need) {
  if (need == 0) need = 1;
  if (*cap >= need) return BDEG_OK;
  if (*ptr) (void)hipFree(*ptr);
  *ptr = nullptr;
  *cap = 0;
  size_t n = need + need / 4;
  if (hipMalloc((void **)ptr, n * sizeof(T)) != hipSuccess) {
    *ptr = nullptr;
    return BDEG_E_NOMEM;
  }
  *cap = n;
  return BDEG_OK;
}

int job_upload(Job &job) {
  int rc;
  if ((rc = grow(&job.d_sys, &job.cap_sys, job.sys.size())) ||
      (rc = grow(&job.d_pts, &job.cap_pts, job.pts.size())) ||
      (rc = grow(&job.d_hts, &job.cap_hts, job.heights.size())) ||
      (rc = grow(&job.d_tiles, &job.cap_tiles, job.tiles.size())))
    return rc;
  static_assert(sizeof(SysAcc) == 32, "SysAcc layout");
  if ((rc = grow(&job.d_acc, &job.cap_acc, job.sys.size()))) return rc;
  if ((rc = grow(&job.d_rerun, &job.cap_rerun, (size_t)RETIE_ROUNDS * (job.sys.size() + 1)))) return rc;
  if (!job.d_cnt && hipMalloc((void **)&job.d_cnt, CNT_BLOCKS * sizeof(DevCounters)) != hipSuccess)
    return BDEG_E_NOMEM;
  if (hipMemcpy(job.d_sys, job.sys.data(), job.sys.size() * sizeof(SysDesc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(job.d_pts, job.pts.data(), job.pts.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(job.d_tiles, job.tiles.data(), job.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess)
    return BDEG_E_DEVICE;
  if (job.explicit_heights &&
      hipMemcpy(job.d_hts, job.heights.data(), job.heights.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
          hipSuccess)
    return BDEG_E_DEVICE;
  return BDEG_OK;
}

int job_launch_pre(Job &job, hipStream_t stream) {
  int rc = launch_clear(stream, job.d_acc, (int)job.sys.size(), job.d_cnt, CNT_BLOCKS);
  if (rc) return rc;
  if (!job.explicit_heights) rc = launch_lift(stream, job.d_sys, nullptr, (int)job.sys.size(), job.d_hts);
  return rc;
}

int job_launch_reset(Job &job, hipStream_t stream) {
  if (job.explicit_heights) return BDEG_E_STATE;
  int rc = launch_reset(stream, job.d_sys, job.d_acc, (int)job.sys.size(), job.d_cnt, CNT_BLOCKS, job.d_rerun,
                        RETIE_ROUNDS);
  if (rc) return rc;
  return launch_lift(stream, job.d_sys, nullptr, (int)job.sys.size(), job.d_hts);
}

int job_launch_retie(Job &job, hipStream_t stream, int round) {
  if (round < 1 || round > RETIE_ROUNDS || job.explicit_heights) return BDEG_E_STATE;
  return launch_retie(stream, job.d_sys, job.d_acc, job.d_hts, (int)job.sys.size(),
                      job.d_rerun + (size_t)(round - 1) * (job.sys.size() + 1));
}

int job_launch_enum(Job &job, hipStream_t stream, int round) {
  if (job.granges.size() > (size_t)MAX_RANGES || round < 0 || round > RETIE_ROUNDS) return BDEG_E_STATE;
  for (size_t i = 0; i < job.granges.size(); i++) {
    const Job::VariantRange &r = job.granges[i];
    LaunchShape shape = job.shape;
    shape.single = r.single;
    shape.dense = r.dense;
    shape.rerun = round ? job.d_rerun + (size_t)(round - 1) * (job.sys.size() + 1) : nullptr;
    int rc = launch_enumerate(stream, job.d_sys, job.d_pts, job.d_hts, job.d_tiles + r.start, r.count, job.d_acc,
                              job.d_cnt + (size_t)round * MAX_RANGES + i, r.klo, r.khi, shape);
    if (rc) return rc;
  }
  return BDEG_OK;
}

int job_launch(Job &job, hipStream_t stream, hipEvent_t e0, hipEvent_t e1) {
  int rc = job_launch_pre(job, stream);
  if (rc) return rc;
  if (e0 && hipEventRecord(e0, stream) != hipSuccess) return BDEG_E_DEVICE;
  if ((rc = job_launch_enum(job, stream))) return rc;
  if (e1 && hipEventRecord(e1, stream) != hipSuccess) return BDEG_E_DEVICE;
  return BDEG_OK;
}

int job_collect(Job &job, hipStream_t stream, std::vector<SysAcc> &acc, DevCounters *cnt) {
  acc.resize(job.sys.size());
  DevCounters blocks[CNT_BLOCKS];
  if (!acc.empty() &&
      hipMemcpyAsync(acc.data(), job.d_acc, acc.size() * sizeof(SysAcc), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return BDEG_E_DEVICE;
  if (hipMemcpyAsync(blocks, job.d_cnt, sizeof(blocks), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return BDEG_E_DEVICE;
  if (hipStreamSynchronize(stream) != hipSuccess) return BDEG_E_DEVICE;
  DevCounters sum{};
  for (const DevCounters &b : blocks) {
    sum.ridges += b.ridges;
    sum.inner += b.inner;
    sum.sp_upd += b.sp_upd;
    sum.pruned += b.pruned;
    sum.leaves += b.leaves;
    sum.rsteps += b.rsteps;
    sum.lsteps += b.lsteps;
    sum.lempty += b.lempty;
    sum.tiles += b.tiles;
    sum.w_inner += b.w_inner;
    sum.w_spatial += b.w_spatial;
    sum.w_ridges += b.w_ridges;
    sum.w_leaves += b.w_leaves;
    sum.triples += b.triples;
    sum.dunits += b.dunits;
    sum.quads += b.quads;
    sum.error |= b.error;
  }
  if (cnt) *cnt = sum;
  if (sum.error) return BDEG_E_DEVICE; // a work unit hit the watchdog
  return BDEG_OK;
}

void Job::release() {
  if (d_sys) (void)hipFree(d_sys);
  if (d_pts) (void)hipFree(d_pts);
  if (d_hts) (void)hipFree(d_hts);
  if (d_tiles) (void)hipFree(d_tiles);
  if (d_acc) (void)hipFree(d_acc);
  if (d_cnt) (void)hipFree(d_cnt);
  if (d_rerun) (void)hipFree(d_rerun);
  d_rerun = nullptr;
  cap_rerun = 0;
  d_sys = nullptr;
  d_pts = nullptr;
  d_hts = nullptr;
  d_tiles = nullptr;
  d_acc = nullptr;
  d_cnt = nullptr;
  cap_sys = cap_pts = cap_hts = cap_tiles = cap_acc = 0;
}

Job::~Job() { release(); }

} // namespace bdeg
