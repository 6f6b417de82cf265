// C-ABI entry points (include/bdeg.h).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "runtime.hpp"

using namespace bdeg;

namespace bdeg {

static bdeg_u128 to_u128(u128 v) { return bdeg_u128{(uint64_t)v, (uint64_t)(v >> 64)}; }

// Host prologue for one input system.  Fills `res` and, when device work is
// needed, `hs` (returns true).
bool prepare_one(const int64_t *A, int m, int n, uint64_t seed, int lift_bits, int index, bdeg_result &res,
                 HostSys &hs) {
  memset(&res, 0, sizeof res);
  if (!A || m < 1 || n < 1 || n > BDEG_MAX_N || lift_bits < 2 || lift_bits > 30) {
    res.status = BDEG_E_ARG;
    return false;
  }
  KernelPoints kp = kernel_points(A, m, n);
  if (kp.status != BDEG_OK) {
    res.status = kp.status;
    return false;
  }
  res.k = kp.k;
  res.rank = kp.rank;
  res.flags = kp.flags;
  res.components = to_u128(kp.comps);
  if (kp.k == 0) {
    res.nvol = bdeg_u128{1, 0};
    res.status = BDEG_OK;
    return false;
  }
  const int N = n + 1;
  if (kp.k > BDEG_MAX_K) {
    res.status = BDEG_E_TOO_LARGE;
    return false;
  }
  uint64_t cand = binom_u64(N, kp.k + 1);
  if (cand >= (1ull << 63)) {
    res.status = BDEG_E_TOO_LARGE;
    return false;
  }
  res.candidates = cand;
  if (!device_bounds_ok(kp.pts.data(), N, kp.k, (1ull << lift_bits) - 1)) {
    res.status = BDEG_E_OVERFLOW;
    return false;
  }
  hs.input_index = index;
  hs.N = N;
  hs.k = kp.k;
  hs.lift_bits = lift_bits;
  hs.attempt = 0;
  hs.seed = seed;
  hs.pts = std::move(kp.pts);
  res.status = BDEG_PENDING;
  return true;
}

int prepare_many(const int64_t *A_concat, const int32_t *m, const int32_t *n, int count, uint64_t seed,
                 int lift_bits, std::vector<bdeg_result> &res, std::vector<HostSys> &dev) {
  res.assign(count, bdeg_result{});
  std::vector<size_t> off(count + 1, 0);
  for (int s = 0; s < count; s++) {
    int64_t mm = m[s], nn = n[s];
    off[s + 1] = off[s] + (size_t)(mm > 0 && nn > 0 ? mm * nn : 0);
  }
  std::vector<HostSys> hs(count);
  std::vector<char> need(count, 0);
  auto work = [&](int lo, int hi) {
    for (int s = lo; s < hi; s++)
      need[s] = prepare_one(A_concat + off[s], m[s], n[s], seed, lift_bits, s, res[s], hs[s]);
  };
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
  if (count < 64) nt = 1;
  std::vector<std::thread> th;
  for (int t = 1; t < nt; t++) th.emplace_back(work, (int)((int64_t)count * t / nt), (int)((int64_t)count * (t + 1) / nt));
  work(0, (int)((int64_t)count / nt));
  for (auto &x : th) x.join();
  dev.clear();
  for (int s = 0; s < count; s++)
    if (need[s]) dev.push_back(std::move(hs[s]));
  return BDEG_OK;
}

// Host plan of the prefix-pruned enumeration (prefixes, unit runs, buckets).
struct PrunePlan {
  int W = 0, d = 0;
  std::vector<uint64_t> items;
  std::vector<uint16_t> chunk_start;
  std::vector<uint8_t> run_lo, run_hi;
  uint32_t off[64] = {0};
  uint64_t cap_units = 0;
};

static int prune_plan(int N, int k, int width, PrunePlan &P);
static int prune_run(Device *D, const PrunePlan &P, const int32_t *points, const int64_t *heights, int N, int k,
                     bdeg_u128 *nvol, int32_t *tie, uint64_t *cells, bdeg_prune_stats *ps);

// The cost model's choice for a one-shot system: the prefix-pruned
// enumeration on the seeded heights of each attempt (drawn on the host by
// the device's own stream), ties redrawn as in the plain path.  Returns
// false, leaving the system to the plain path, when the model or the
// pruned path's limits say no; a device error is reported in *rc.
static bool solve_pruned(Device *D, HostSys &h, bdeg_result &r, int *rc) {
  *rc = BDEG_OK;
  if (schedule_mode() != BDEG_SCHED_AUTO || binom_u64(h.N, h.k + 1) < BDEG_PRUNE_MIN_CANDIDATES) return false;
  PrunePlan P;
  if (prune_plan(h.N, h.k, 0, P) != BDEG_OK) return false;
  std::vector<int64_t> hts((size_t)h.N);
  for (;;) {
    const uint64_t key = lift_key(h.seed, 0, h.attempt);
    for (int j = 0; j < h.N; j++) hts[(size_t)j] = lift_height(key, j, h.lift_bits);
    if (h.attempt == 0 && check_points(h.pts.data(), hts.data(), h.N, h.k) != BDEG_OK) return false;
    bdeg_u128 nv{0, 0};
    int32_t tie = 0;
    uint64_t cells = 0;
    if ((*rc = prune_run(D, P, h.pts.data(), hts.data(), h.N, h.k, &nv, &tie, &cells, nullptr))) return true;
    r.attempts = (int32_t)h.attempt + 1;
    r.flags |= BDEG_F_PRUNED;
    if (!tie) {
      r.nvol = nv;
      r.cells = cells;
      r.status = BDEG_OK;
      return true;
    }
    if (h.attempt + 1 >= (uint32_t)BDEG_MAX_ATTEMPTS) {
      r.status = BDEG_E_TIE;
      return true;
    }
    h.attempt++;
  }
}

// Run device systems to completion: tie retries redraw the lifting of the
// tied systems only.  `first` (optional) is an already-launched job holding
// all of `dev` in order; without it, systems the cost model picks run the
// prefix-pruned enumeration instead (solve_pruned).
int finish_device(Device *D, std::vector<HostSys> &dev, std::vector<bdeg_result> &res, Job *first,
                  DevCounters *cnt_out, int32_t *redraws_out) {
  std::vector<int> pending;
  for (size_t i = 0; i < dev.size(); i++) {
    if (!first) {
      int rc = BDEG_OK;
      if (solve_pruned(D, dev[i], res[dev[i].input_index], &rc)) {
        if (rc) return rc;
        continue;
      }
    }
    pending.push_back((int)i);
  }
  Job local;
  for (int round = 0; !pending.empty(); round++) {
    Job *job = (round == 0 && first) ? first : &local;
    std::vector<HostSys> subset;
    if (!(round == 0 && first)) {
      for (int i : pending) subset.push_back(dev[i]);
      uint64_t total = 0;
      int kmax = 1, kmin = 64;
      for (auto &h : subset) {
        total += binom_u64(h.N, h.k + 1);
        kmax = std::max(kmax, h.k);
        kmin = std::min(kmin, h.k);
      }
      job_build_seeded(*job, subset, choose_max_cost(total, default_waves(std::min(kmin, kmax), kmax, 4)));
      int rc = job_upload(*job);
      if (rc) return rc;
      rc = job_launch(*job, D->stream);
      if (rc) return rc;
    }
    std::vector<SysAcc> acc;
    DevCounters cnt;
    int rc = job_collect(*job, D->stream, acc, &cnt);
    if (rc) return rc;
    if (round == 0 && cnt_out) *cnt_out = cnt;
    if (round == 0 && redraws_out) {
      int32_t n = 0;
      for (const SysAcc &a : acc) n += a.attempt > 0;
      *redraws_out = n;
    }
    std::vector<int> next;
    for (size_t q = 0; q < pending.size(); q++) {
      HostSys &h = dev[pending[q]];
      bdeg_result &r = res[h.input_index];
      // draws made inside the device pass (a prepared batch's redraw rounds)
      // come on top of the host's
      const uint32_t att = h.attempt + acc[q].attempt;
      r.attempts = (int32_t)att + 1;
      if (acc[q].tie) {
        if (att + 1 >= BDEG_MAX_ATTEMPTS) {
          r.status = BDEG_E_TIE;
          continue;
        }
        h.attempt = att + 1;
        next.push_back(pending[q]);
        continue;
      }
      r.nvol = bdeg_u128{acc[q].lo, acc[q].hi};
      r.cells = acc[q].cells;
      r.status = BDEG_OK;
    }
    pending.swap(next);
  }
  return BDEG_OK;
}

int check_points(const int32_t *points, const int64_t *heights, int N, int k) {
  if (!points || !heights || k < 1 || k > BDEG_MAX_K || N < k + 1 || N > 64) return BDEG_E_ARG;
  int64_t hmin = heights[0], hmax = heights[0];
  for (int j = 0; j < N; j++) {
    if (heights[j] >= (1ll << 40) || heights[j] <= -(1ll << 40)) return BDEG_E_ARG;
    hmin = std::min(hmin, heights[j]);
    hmax = std::max(hmax, heights[j]);
  }
  if (!device_bounds_ok(points, N, k, (uint64_t)(hmax - hmin))) return BDEG_E_OVERFLOW;
  return BDEG_OK;
}

// One caller point set with explicit heights, candidates of colex rank in [rank_lo, rank_hi).
void points_job(Job &job, const int32_t *points, const int64_t *heights, int N, int k, uint64_t rank_lo,
                uint64_t rank_hi, uint64_t max_cost) {
  job.sys.clear();
  job.tiles.clear();
  SysDesc d;
  d.N = N;
  d.k = k;
  d.pt_off = 0;
  d.ht_off = 0;
  d.lift_bits = 0;
  d.npad_log2 = npad_log2_for(N);
  d.lift_key = 0;
  d.seed = 0;
  d.sys_index = 0;
  int64_t hmin = heights[0], hmax = heights[0];
  for (int j = 1; j < N; j++) {
    hmin = std::min(hmin, heights[j]);
    hmax = std::max(hmax, heights[j]);
  }
  d.flags = dense_ok(points, N, k, (uint64_t)(hmax - hmin)) ? SYS_DENSE : 0;
  job.sys.push_back(d);
  job.pts.assign(points, points + (size_t)N * k);
  job.heights.assign(heights, heights + N);
  job.explicit_heights = true;
  job.kmin = job.kmax = k;
  const uint64_t total = binom_u64(N, k + 1);
  const uint64_t hi = std::min(rank_hi, total), lo = std::min(rank_lo, hi);
  if (lo == 0 && hi == total && total > 0) job.sys[0].flags |= SYS_SORTED; // every candidate: may relabel
  std::vector<TileC> tc;
  tiles_range(N, k, 0, lo, hi, max_cost ? max_cost : choose_max_cost(hi - lo, default_waves(k, k, 4)), tc);
  job_order_units(job, tc);
}

// Device buffers of one cell listing, freed on scope exit.
struct CellBuffers {
  uint64_t *masks = nullptr, *den = nullptr, *count = nullptr;
  int64_t *num = nullptr;
  uint32_t *err = nullptr;
  int alloc(uint64_t cap, int k) {
    if (cap > (1ull << 40) / (8ull * (k + 2))) return BDEG_E_NOMEM;
    if (hipMalloc((void **)&count, sizeof(uint64_t)) != hipSuccess ||
        hipMalloc((void **)&err, sizeof(uint32_t)) != hipSuccess)
      return BDEG_E_NOMEM;
    if (cap > 0 && (hipMalloc((void **)&masks, cap * sizeof(uint64_t)) != hipSuccess ||
                    hipMalloc((void **)&den, cap * sizeof(uint64_t)) != hipSuccess ||
                    hipMalloc((void **)&num, cap * (size_t)k * sizeof(int64_t)) != hipSuccess))
      return BDEG_E_NOMEM;
    return BDEG_OK;
  }
  ~CellBuffers() {
    for (void *p : {(void *)masks, (void *)den, (void *)count, (void *)num, (void *)err})
      if (p) (void)hipFree(p);
  }
};

// Enumerate an uploaded one-system job with the cell-listing kernel variant,
// then compute the inner normals of the stored cells; copies out at most cap
// cells, *n_cells = all found, *acc_out = the system's accumulator.
static int list_cells(Device *D, Job &job, int N, int k, uint64_t cap, uint64_t *masks, int64_t *num,
                      uint64_t *den, uint64_t *n_cells, SysAcc *acc_out) {
  CellBuffers b;
  int rc = b.alloc(cap, k);
  if (rc) return rc;
  if (hipMemsetAsync(b.count, 0, sizeof(uint64_t), D->stream) != hipSuccess ||
      hipMemsetAsync(b.err, 0, sizeof(uint32_t), D->stream) != hipSuccess)
    return BDEG_E_DEVICE;
  job.shape.mode = MODE_EMIT;
  job.shape.sink = CellSink{b.masks, cap, b.count};
  rc = job_launch(job, D->stream);
  job.shape.mode = MODE_PLAIN;
  job.shape.sink = CellSink{nullptr, 0, nullptr};
  if (rc) return rc;
  std::vector<SysAcc> acc;
  rc = job_collect(job, D->stream, acc, nullptr);
  if (rc) return rc;
  uint64_t count = 0;
  if (hipMemcpyAsync(&count, b.count, sizeof count, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
      hipStreamSynchronize(D->stream) != hipSuccess)
    return BDEG_E_DEVICE;
  if (count != acc[0].cells) return BDEG_E_DEVICE; // every accepted facet is listed exactly once
  const uint64_t stored = std::min(count, cap);
  rc = launch_cell_normals(D->stream, b.masks, stored, job.d_pts, job.d_hts, N, k, b.num, b.den, b.err);
  if (rc) return rc;
  uint32_t err = 0;
  if (hipMemcpyAsync(&err, b.err, sizeof err, hipMemcpyDeviceToHost, D->stream) != hipSuccess) return BDEG_E_DEVICE;
  if (stored > 0 &&
      (hipMemcpyAsync(masks, b.masks, stored * sizeof(uint64_t), hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
       hipMemcpyAsync(num, b.num, stored * (size_t)k * sizeof(int64_t), hipMemcpyDeviceToHost, D->stream) !=
           hipSuccess ||
       hipMemcpyAsync(den, b.den, stored * sizeof(uint64_t), hipMemcpyDeviceToHost, D->stream) != hipSuccess))
    return BDEG_E_DEVICE;
  if (hipStreamSynchronize(D->stream) != hipSuccess) return BDEG_E_DEVICE;
  if (err & 1u) return BDEG_E_DEVICE;   // a listed mask is not a (k+1)-subset
  if (err & 2u) return BDEG_E_OVERFLOW; // a value outside the certified widths
  *n_cells = count;
  *acc_out = acc[0];
  return BDEG_OK;
}

static int first_error(const std::vector<bdeg_result> &res) {
  for (auto &r : res)
    if (r.status != BDEG_OK) return r.status;
  return BDEG_OK;
}

} // namespace bdeg

struct bdeg_batch {
  std::vector<bdeg_result> res;
  std::vector<HostSys> dev;
  Job job;
  // the device pass is three captured graphs: reset + lift, the enumeration
  // (HIP events between them time the enumeration alone), and the redraw
  // rounds of tied systems (each a no-op launch when nothing tied)
  hipGraph_t graph_pre = nullptr, graph_enum = nullptr, graph_retry = nullptr;
  hipGraphExec_t exec_pre = nullptr, exec_enum = nullptr, exec_retry = nullptr;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr, ev_k0 = nullptr, ev_k1 = nullptr;
  bool launched = false;
  bdeg_stats stats{};
};

namespace bdeg {

static void batch_drop_graphs(bdeg_batch *b) {
  for (hipGraphExec_t x : {b->exec_pre, b->exec_enum, b->exec_retry})
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t g : {b->graph_pre, b->graph_enum, b->graph_retry})
    if (g) (void)hipGraphDestroy(g);
  b->exec_pre = b->exec_enum = b->exec_retry = nullptr;
  b->graph_pre = b->graph_enum = b->graph_retry = nullptr;
  b->stats.captured = 0;
}

// Work units for the batch's systems (with a tuned schedule when given),
// upload, and capture the device pass (reset + lift; enumeration; redraw
// rounds) as three graphs.  Called with the device mutex held.
static int batch_setup(bdeg_batch *b, Device *D, const ScheduleTable *sched) {
  batch_drop_graphs(b);
  if (b->dev.empty()) return BDEG_OK;
  uint64_t total = 0;
  int kmax = 1, kmin = 64;
  for (auto &h : b->dev) {
    total += binom_u64(h.N, h.k + 1);
    kmax = std::max(kmax, h.k);
    kmin = std::min(kmin, h.k);
  }
  job_build_seeded(b->job, b->dev, choose_max_cost(total, default_waves(std::min(kmin, kmax), kmax, 4)), sched);
  int rc = job_upload(b->job);
  if (rc) return rc;
  auto capture = [&](int part, hipGraph_t *g, hipGraphExec_t *x) {
    if (hipStreamBeginCapture(D->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    int rc2 = BDEG_OK;
    if (part == 0) rc2 = job_launch_reset(b->job, D->stream);
    else if (part == 1) rc2 = job_launch_enum(b->job, D->stream, 0);
    else
      for (int r = 1; r <= RETIE_ROUNDS && rc2 == BDEG_OK; r++)
        if (!(rc2 = job_launch_retie(b->job, D->stream, r))) rc2 = job_launch_enum(b->job, D->stream, r);
    hipGraph_t gg = nullptr;
    hipError_t e = hipStreamEndCapture(D->stream, &gg);
    if (rc2 == BDEG_OK && e == hipSuccess && gg && hipGraphInstantiate(x, gg, nullptr, nullptr, 0) == hipSuccess) {
      *g = gg;
      return true;
    }
    if (gg) (void)hipGraphDestroy(gg);
    *x = nullptr;
    (void)hipGetLastError();
    return false;
  };
  if (capture(0, &b->graph_pre, &b->exec_pre) && capture(1, &b->graph_enum, &b->exec_enum) &&
      capture(2, &b->graph_retry, &b->exec_retry))
    b->stats.captured = 1;
  else
    batch_drop_graphs(b); // the same pass then runs as plain launches (stats.captured == 0)
  return BDEG_OK;
}

// Device time of the first enumeration of `systems` alone under `sched`
// (median of `reps` timed passes after one warm-up); the volume sums of the
// pass are returned for the tuner's consistency check.
static int time_schedule(Device *D, const std::vector<HostSys> &systems, const ScheduleTable *sched, int reps,
                         float *ms, std::vector<SysAcc> *sums) {
  Job job;
  uint64_t total = 0;
  int kmax = 1, kmin = 64;
  for (auto &h : systems) {
    total += binom_u64(h.N, h.k + 1);
    kmax = std::max(kmax, h.k);
    kmin = std::min(kmin, h.k);
  }
  job_build_seeded(job, systems, choose_max_cost(total, default_waves(std::min(kmin, kmax), kmax, 4)), sched);
  int rc = job_upload(job);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return BDEG_E_DEVICE;
  }
  std::vector<float> t;
  for (int r = 0; r <= reps && !rc; r++) {
    rc = job_launch_reset(job, D->stream);
    if (!rc && hipEventRecord(e0, D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
    if (!rc) rc = job_launch_enum(job, D->stream, 0);
    if (!rc && hipEventRecord(e1, D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
    if (!rc) rc = job_collect(job, D->stream, *sums, nullptr);
    float x = 0;
    if (!rc && r > 0 && hipEventElapsedTime(&x, e0, e1) == hipSuccess) t.push_back(x);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  std::sort(t.begin(), t.end());
  *ms = t.empty() ? 0.f : t[t.size() / 2];
  return BDEG_OK;
}

} // namespace bdeg

extern "C" {

int bdeg_init(int32_t device) { return device_select(device); }

const char *bdeg_strerror(int code) {
  switch (code) {
    case BDEG_OK: return "ok";
    case BDEG_PENDING: return "pending";
    case BDEG_E_ARG: return "invalid argument";
    case BDEG_E_OVERFLOW: return "integer bound exceeded (host int64 algebra or device minor bound)";
    case BDEG_E_TOO_LARGE: return "problem too large (k above the device limit or too many candidates)";
    case BDEG_E_TIE: return "no generic lifting found";
    case BDEG_E_DEVICE: return "HIP device error or no device";
    case BDEG_E_NOMEM: return "out of memory";
    case BDEG_E_STATE: return "invalid state";
    default: return "unknown error";
  }
}

int bdeg_kernel_points(const int64_t *A, int32_t m, int32_t n, int32_t *k, int32_t *rank, bdeg_u128 *components,
                       int32_t *points) {
  if (!A || !k || !rank || !components || !points || m < 1 || n < 1 || n > BDEG_MAX_N) return BDEG_E_ARG;
  KernelPoints kp = kernel_points(A, m, n);
  if (kp.status != BDEG_OK) return kp.status;
  *k = kp.k;
  *rank = kp.rank;
  *components = to_u128(kp.comps);
  if (!kp.pts.empty()) memcpy(points, kp.pts.data(), kp.pts.size() * sizeof(int32_t));
  return BDEG_OK;
}

int bdeg_consistency(const int64_t *A, int32_t m, int32_t n, const double *b, double tol, int32_t *consistent,
                     double *residual, int32_t *relations) {
  if (!A || !b || !consistent || !residual || !relations || m < 1 || n < 1 || n > BDEG_MAX_N || m > 4096 ||
      !(tol >= 0))
    return BDEG_E_ARG;
  for (int i = 0; i < m; i++)
    if (b[2 * i] == 0.0 && b[2 * i + 1] == 0.0) return BDEG_E_ARG;
  // left kernel of A = integer kernel of A^T (n x m)
  std::vector<int64_t> At((size_t)n * m);
  for (int i = 0; i < m; i++)
    for (int j = 0; j < n; j++) At[(size_t)j * m + i] = A[(size_t)i * n + j];
  KernelPoints kp = kernel_points(At.data(), n, m);
  if (kp.status != BDEG_OK) return kp.status;
  const int rel = kp.k; // m - rank
  double worst = 0.0;
  for (int c = 0; c < rel; c++) {
    std::complex<double> prod(1.0, 0.0);
    for (int i = 0; i < m; i++) {
      const int64_t q = kp.pts[(size_t)(i + 1) * rel + c];
      if (q == 0) continue;
      std::complex<double> base(b[2 * i], b[2 * i + 1]);
      if (q < 0) base = 1.0 / base;
      uint64_t e = (uint64_t)(q < 0 ? -q : q);
      std::complex<double> pw(1.0, 0.0);
      while (e) {
        if (e & 1) pw *= base;
        base *= base;
        e >>= 1;
      }
      prod *= pw;
    }
    worst = std::max(worst, std::abs(prod - 1.0));
  }
  *relations = rel;
  *residual = worst;
  *consistent = worst <= tol ? 1 : 0;
  return BDEG_OK;
}

int bdeg_degree_batch(const int64_t *A_concat, const int32_t *m, const int32_t *n, int32_t count, uint64_t seed,
                      int32_t lift_bits, bdeg_result *out) {
  if (!A_concat || !m || !n || !out || count < 1) return BDEG_E_ARG;
  std::vector<bdeg_result> res;
  std::vector<HostSys> dev;
  prepare_many(A_concat, m, n, count, seed, lift_bits, res, dev);
  if (!dev.empty()) {
    int st;
    Device *D = device_get(&st);
    if (!D) {
      for (auto &h : dev) res[h.input_index].status = st;
    } else {
      std::lock_guard<std::mutex> lk(D->mu);
      int rc = finish_device(D, dev, res, nullptr, nullptr);
      if (rc)
        for (auto &h : dev)
          if (res[h.input_index].status == BDEG_PENDING) res[h.input_index].status = rc;
    }
  }
  memcpy(out, res.data(), res.size() * sizeof(bdeg_result));
  return first_error(res);
}

int bdeg_set_schedule(int32_t schedule) { return schedule_set(schedule); }

int bdeg_degree(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits, bdeg_result *out) {
  if (!A || !out) return BDEG_E_ARG;
  return bdeg_degree_batch(A, &m, &n, 1, seed, lift_bits, out);
}

int bdeg_batch_create(const int64_t *A_concat, const int32_t *m, const int32_t *n, int32_t count, uint64_t seed,
                      int32_t lift_bits, bdeg_batch **out) {
  if (!A_concat || !m || !n || !out || count < 1) return BDEG_E_ARG;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  bdeg_batch *b = new bdeg_batch();
  prepare_many(A_concat, m, n, count, seed, lift_bits, b->res, b->dev);
  std::lock_guard<std::mutex> lk(D->mu);
  if (hipEventCreate(&b->ev_t0) != hipSuccess || hipEventCreate(&b->ev_t1) != hipSuccess ||
      hipEventCreate(&b->ev_k0) != hipSuccess || hipEventCreate(&b->ev_k1) != hipSuccess) {
    delete b;
    return BDEG_E_DEVICE;
  }
  const ScheduleTable &tab = schedule_table();
  const int rc = batch_setup(b, D, tab.any ? &tab : nullptr);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return BDEG_OK;
}

int bdeg_batch_run(bdeg_batch *b) {
  if (!b) return BDEG_E_ARG;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  if (b->dev.empty()) {
    b->launched = true;
    return BDEG_OK;
  }
  std::lock_guard<std::mutex> lk(D->mu);
  // every run starts from attempt 0 (same liftings as the captured graph)
  for (auto &h : b->dev) h.attempt = 0;
  if (hipEventRecord(b->ev_t0, D->stream) != hipSuccess) return BDEG_E_DEVICE;
  if (b->stats.captured) {
    if (hipGraphLaunch(b->exec_pre, D->stream) != hipSuccess) return BDEG_E_DEVICE;
    if (hipEventRecord(b->ev_k0, D->stream) != hipSuccess) return BDEG_E_DEVICE;
    if (hipGraphLaunch(b->exec_enum, D->stream) != hipSuccess) return BDEG_E_DEVICE;
    if (hipEventRecord(b->ev_k1, D->stream) != hipSuccess) return BDEG_E_DEVICE;
    if (hipGraphLaunch(b->exec_retry, D->stream) != hipSuccess) return BDEG_E_DEVICE;
  } else {
    // the same pass as plain launches (capture was refused by the runtime)
    int rc = job_launch_reset(b->job, D->stream);
    if (!rc && hipEventRecord(b->ev_k0, D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
    if (!rc) rc = job_launch_enum(b->job, D->stream, 0);
    if (!rc && hipEventRecord(b->ev_k1, D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
    for (int r = 1; r <= RETIE_ROUNDS && !rc; r++)
      if (!(rc = job_launch_retie(b->job, D->stream, r))) rc = job_launch_enum(b->job, D->stream, r);
    if (rc) return rc;
  }
  if (hipEventRecord(b->ev_t1, D->stream) != hipSuccess) return BDEG_E_DEVICE;
  b->launched = true;
  return BDEG_OK;
}

int bdeg_batch_results(bdeg_batch *b, bdeg_result *out) {
  if (!b || !out) return BDEG_E_ARG;
  if (!b->launched) return BDEG_E_STATE;
  if (!b->dev.empty()) {
    int st;
    Device *D = device_get(&st);
    if (!D) return st;
    std::lock_guard<std::mutex> lk(D->mu);
    if (hipEventSynchronize(b->ev_t1) != hipSuccess) return BDEG_E_DEVICE;
    float t = 0, k = 0;
    (void)hipEventElapsedTime(&t, b->ev_t0, b->ev_t1);
    (void)hipEventElapsedTime(&k, b->ev_k0, b->ev_k1);
    int rc = finish_device(D, b->dev, b->res, &b->job, nullptr, &b->stats.redraws);
    if (rc) return rc;
    b->stats.kernel_ms = k;
    b->stats.total_ms = t;
  }
  b->launched = false;
  memcpy(out, b->res.data(), b->res.size() * sizeof(bdeg_result));
  return first_error(b->res);
}

int bdeg_batch_stats(const bdeg_batch *b, bdeg_stats *out) {
  if (!b || !out) return BDEG_E_ARG;
  *out = b->stats;
  return BDEG_OK;
}

int bdeg_batch_profile(bdeg_batch *b) {
  if (!b) return BDEG_E_ARG;
  if (b->dev.empty()) return BDEG_OK;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  // the first enumeration of the pass (attempt-0 liftings), counting its work
  b->job.shape.mode = MODE_STATS;
  int rc = job_launch_reset(b->job, D->stream);
  if (!rc) rc = job_launch_enum(b->job, D->stream, 0);
  b->job.shape.mode = MODE_PLAIN;
  if (rc) return rc;
  std::vector<SysAcc> acc;
  DevCounters cnt{};
  rc = job_collect(b->job, D->stream, acc, &cnt);
  if (rc) return rc;
  b->stats.ridges = cnt.ridges;
  b->stats.inner_nodes = cnt.inner;
  b->stats.spatial_updates = cnt.sp_upd;
  b->stats.pruned = cnt.pruned;
  b->stats.leaves = cnt.leaves;
  b->stats.ridge_steps = cnt.rsteps;
  b->stats.leaf_steps = cnt.lsteps;
  b->stats.empty_steps = cnt.lempty;
  b->stats.tiles = cnt.tiles;
  b->stats.point_inner = cnt.w_inner;
  b->stats.point_spatial = cnt.w_spatial;
  b->stats.point_ridges = cnt.w_ridges;
  b->stats.leaf_points = cnt.w_leaves;
  b->stats.triples = cnt.triples;
  b->stats.dense_units = cnt.dunits;
  b->stats.quads = cnt.quads;
  return BDEG_OK;
}

int bdeg_batch_tune(bdeg_batch *b, const char *table_path, int32_t reps) {
  if (!b || reps < 1 || reps > 64) return BDEG_E_ARG;
  if (b->dev.empty()) return BDEG_OK;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  // buckets of the batch: (k, smallest lane-group width)
  std::vector<HostSys> bucket[BDEG_MAX_K + 1][7];
  for (auto &h : b->dev) {
    HostSys c = h;
    c.attempt = 0;
    bucket[h.k][npad_log2_for(h.N)].push_back(c);
  }
  ScheduleTable best;
  if (table_path) (void)schedule_read(table_path, best); // keep other buckets' entries
  static const uint64_t COSTS[] = {128, 256, 512, 1024, 2048, 4096, 8192};
  for (int k = 1; k <= BDEG_MAX_K; k++)
    for (int g = 3; g <= 6; g++) {
      const std::vector<HostSys> &sys = bucket[k][g];
      if (sys.empty()) continue;
      // the default schedule first: its sums are the reference every other
      // schedule must reproduce exactly (same liftings, same candidates)
      std::vector<SysAcc> ref, sums;
      float ms_best = 0;
      int rc = time_schedule(D, sys, nullptr, reps, &ms_best, &ref);
      if (rc) return rc;
      BucketSchedule pick;
      pick.ms = ms_best;
      // the kernel: lanes as points at the smallest or the next lane-group
      // width, or lane-dense (for the systems it is certified for; the group
      // width does not apply); each at every unit size
      for (int dense = 0; dense <= 1; dense++)
        for (int w = g; w <= (dense ? g : std::min(6, g + 1)); w++)
          for (uint64_t cost : COSTS) {
            ScheduleTable one;
            one.e[k][g].dense = dense;
            one.e[k][g].npad_log2 = w;
            one.e[k][g].unit_cost = cost;
            one.any = true;
            float ms = 0;
            rc = time_schedule(D, sys, &one, reps, &ms, &sums);
            if (rc) return rc;
            for (size_t i = 0; i < ref.size(); i++)
              if (sums[i].lo != ref[i].lo || sums[i].hi != ref[i].hi || sums[i].cells != ref[i].cells ||
                  sums[i].tie != ref[i].tie)
                return BDEG_E_STATE; // a schedule changed a result: never persist it
            if (ms < pick.ms) {
              pick.ms = ms;
              pick.dense = dense;
              pick.npad_log2 = w;
              pick.unit_cost = cost;
            }
          }
      pick.systems = (int)sys.size();
      if (pick.npad_log2 == 0) { // the default won: record it explicitly
        pick.npad_log2 = g;
        pick.unit_cost = 0;
      }
      best.e[k][g] = pick;
      best.any = true;
    }
  if (table_path) {
    const int rc = schedule_write(table_path, best);
    if (rc) return rc;
  }
  return batch_setup(b, D, &best);
}

int bdeg_batch_destroy(bdeg_batch *b) {
  if (!b) return BDEG_E_ARG;
  int st;
  Device *D = device_get(&st);
  if (D) {
    std::lock_guard<std::mutex> lk(D->mu);
    (void)hipStreamSynchronize(D->stream);
    for (hipGraphExec_t x : {b->exec_pre, b->exec_enum, b->exec_retry})
      if (x) (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : {b->graph_pre, b->graph_enum, b->graph_retry})
      if (g) (void)hipGraphDestroy(g);
    if (b->ev_t0) (void)hipEventDestroy(b->ev_t0);
    if (b->ev_t1) (void)hipEventDestroy(b->ev_t1);
    if (b->ev_k0) (void)hipEventDestroy(b->ev_k0);
    if (b->ev_k1) (void)hipEventDestroy(b->ev_k1);
    b->job.release();
  }
  delete b;
  return BDEG_OK;
}

int bdeg_nvol_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t rank_lo,
                     uint64_t rank_hi, bdeg_u128 *nvol, int32_t *tie, uint64_t *cells) {
  if (!nvol || !tie) return BDEG_E_ARG;
  int rc = check_points(points, heights, N, k);
  if (rc) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  static Job job; // scratch job reused across calls (guarded by the device mutex)
  points_job(job, points, heights, N, k, rank_lo, rank_hi);
  rc = job_upload(job);
  if (rc) return rc;
  rc = job_launch(job, D->stream);
  if (rc) return rc;
  std::vector<SysAcc> acc;
  rc = job_collect(job, D->stream, acc, nullptr);
  if (rc) return rc;
  *nvol = bdeg_u128{acc[0].lo, acc[0].hi};
  *tie = (int32_t)acc[0].tie;
  if (cells) *cells = acc[0].cells;
  return BDEG_OK;
}

namespace bdeg {

static int prune_plan(int N, int k, int width, PrunePlan &P) {
  // prefix states with W free columns: W = width, or 5 widened while there
  // are more than 2^18 prefixes (the tests then cost more than they save)
  int &W = P.W;
  W = width > 0 ? width : std::min(k, 5);
  if (W < 1 || W > PRUNE_WMAX || W > k) return BDEG_E_ARG;
  if (width <= 0)
    while (W < PRUNE_WMAX && W < k && binom_u64(N - W, k + 1 - W) > (1ull << 18)) W++;
  const int d = P.d = k + 1 - W; // prefix size; its lowest element is >= W
  const uint64_t n_items = binom_u64(N - W, d);
  if (n_items > BDEG_PRUNE_MAX_PREFIXES) return BDEG_E_TOO_LARGE;
  // the prefixes: d-subsets of {W, .., N-1}; each kept one gives e - W + 1 units
  std::vector<uint64_t> &items = P.items;
  items.reserve((size_t)n_items);
  // d-subsets of {0, .., N-W-1} in increasing order (Gosper), shifted up by W;
  // a prefix with lowest point e gives one unit for each next element
  // c = W-1 .. e-1, which goes to bucket c
  uint64_t per_c[64] = {0};
  const uint64_t lim = (1ull << (N - W)) - 1; // N - W < 64
  for (uint64_t m = (1ull << d) - 1; m <= lim;) {
    items.push_back(m << W);
    per_c[__builtin_ctzll(m) + W]++; // prefixes with lowest point e = ctz + W
    const uint64_t c = m & (0 - m), r = m + c;
    m = (((r ^ m) >> 2) / c) | r;
  }
  // chunk c: the subtree of F + c split into runs of the following element
  // (each run at most the plain plan's unit cost); one run [c, c] when F + c
  // is already a whole candidate (W = 1)
  const uint64_t max_cost = choose_max_cost(binom_u64(N, k + 1), default_waves(k, k, 4));
  std::vector<uint16_t> &chunk_start = P.chunk_start;
  chunk_start.assign(65, 0);
  std::vector<uint8_t> &run_lo = P.run_lo, &run_hi = P.run_hi;
  for (int c = 0; c < 64; c++) {
    chunk_start[c] = (uint16_t)run_lo.size();
    if (c < W - 1 || c >= N) continue;
    if (W == 1) {
      run_lo.push_back((uint8_t)c);
      run_hi.push_back((uint8_t)c);
      continue;
    }
    // element after c: c2 in [W-2, c-1], C(c2, W-2) candidates each
    int hi = c - 1;
    while (hi >= W - 2) {
      int lo = hi;
      uint64_t cost = binom_u64(hi, W - 2);
      while (lo - 1 >= W - 2 && cost + binom_u64(lo - 1, W - 2) <= max_cost) cost += binom_u64(--lo, W - 2);
      run_lo.push_back((uint8_t)lo);
      run_hi.push_back((uint8_t)hi);
      hi = lo - 1;
    }
  }
  chunk_start[64] = (uint16_t)run_lo.size();
  if (run_lo.empty()) return BDEG_E_TOO_LARGE;
  // bucket c holds chunk c of every prefix with e > c; laid out from c = N-1 down
  uint32_t *off = P.off;
  uint64_t &cap_units = P.cap_units, above = 0;
  for (int c = N - 1; c >= W - 1; c--) {
    off[c] = (uint32_t)std::min<uint64_t>(cap_units, 0xFFFFFFFFull);
    cap_units += above * (uint64_t)(chunk_start[c + 1] - chunk_start[c]); // prefixes whose lowest point is above c
    above += per_c[c];
  }
  if (cap_units == 0 || cap_units > 0xFFFFFFFFull) return BDEG_E_TOO_LARGE;
  return BDEG_OK;
}

// Device part of the prefix-pruned enumeration (the device lock held).
static int prune_run(Device *D, const PrunePlan &P, const int32_t *points, const int64_t *heights, int N, int k,
                     bdeg_u128 *nvol, int32_t *tie, uint64_t *cells, bdeg_prune_stats *ps) {
  const int W = P.W, d = P.d;
  const std::vector<uint64_t> &items = P.items;
  const std::vector<uint16_t> &chunk_start = P.chunk_start;
  const std::vector<uint8_t> &run_lo = P.run_lo, &run_hi = P.run_hi;
  const uint32_t *off = P.off;
  const uint64_t cap_units = P.cap_units;
  int rc = BDEG_OK;
  Job job;
  points_job(job, points, heights, N, k, 0, 0); // no units: they come from the prefixes
  if ((rc = job_upload(job)) || (rc = job_launch_pre(job, D->stream))) return rc;
  uint64_t *d_items = nullptr;
  Tile *d_raw = nullptr, *d_units = nullptr;
  PruneCounters *d_pc = nullptr;
  uint32_t *d_off = nullptr, *d_bcnt = nullptr;
  uint16_t *d_cs = nullptr;
  uint8_t *d_rlo = nullptr, *d_rhi = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  auto cleanup = [&]() {
    if (d_items) (void)hipFree(d_items);
    if (d_raw) (void)hipFree(d_raw);
    if (d_units) (void)hipFree(d_units);
    if (d_pc) (void)hipFree(d_pc);
    if (d_off) (void)hipFree(d_off);
    if (d_bcnt) (void)hipFree(d_bcnt);
    if (d_cs) (void)hipFree(d_cs);
    if (d_rlo) (void)hipFree(d_rlo);
    if (d_rhi) (void)hipFree(d_rhi);
    for (hipEvent_t &e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (hipMalloc((void **)&d_items, items.size() * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc((void **)&d_raw, cap_units * sizeof(Tile)) != hipSuccess ||
      hipMalloc((void **)&d_units, cap_units * sizeof(Tile)) != hipSuccess ||
      hipMalloc((void **)&d_pc, sizeof(PruneCounters)) != hipSuccess ||
      hipMalloc((void **)&d_off, 64 * sizeof(uint32_t)) != hipSuccess || hipMalloc((void **)&d_bcnt, 64 * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc((void **)&d_cs, chunk_start.size() * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc((void **)&d_rlo, run_lo.size()) != hipSuccess || hipMalloc((void **)&d_rhi, run_hi.size()) != hipSuccess) {
    cleanup();
    return BDEG_E_NOMEM;
  }
  PruneCounters pc{};
  for (hipEvent_t &e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      cleanup();
      return BDEG_E_DEVICE;
    }
  if (hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(uint64_t), hipMemcpyHostToDevice, D->stream) !=
          hipSuccess ||
      hipMemcpyAsync(d_pc, &pc, sizeof pc, hipMemcpyHostToDevice, D->stream) != hipSuccess ||
      hipMemcpyAsync(d_off, off, 64 * sizeof(uint32_t), hipMemcpyHostToDevice, D->stream) != hipSuccess ||
      hipMemsetAsync(d_bcnt, 0, 64 * sizeof(uint32_t), D->stream) != hipSuccess ||
      hipMemcpyAsync(d_cs, chunk_start.data(), chunk_start.size() * sizeof(uint16_t), hipMemcpyHostToDevice,
                     D->stream) != hipSuccess ||
      hipMemcpyAsync(d_rlo, run_lo.data(), run_lo.size(), hipMemcpyHostToDevice, D->stream) != hipSuccess ||
      hipMemcpyAsync(d_rhi, run_hi.data(), run_hi.size(), hipMemcpyHostToDevice, D->stream) != hipSuccess ||
      hipEventRecord(ev[0], D->stream) != hipSuccess) {
    cleanup();
    return BDEG_E_DEVICE;
  }
  PruneArgs a;
  a.pts = job.d_pts;
  a.hts = job.d_hts;
  a.N = N;
  a.K = k;
  a.W = W;
  a.items = d_items;
  a.n_items = (uint32_t)items.size();
  a.units = d_raw;
  a.cap_units = (uint32_t)cap_units;
  a.bucket_off = d_off;
  a.bucket_cnt = d_bcnt;
  a.chunk_start = d_cs;
  a.run_lo = d_rlo;
  a.run_hi = d_rhi;
  a.cnt = d_pc;
  uint32_t bcnt[64] = {0};
  rc = launch_prune(D->stream, a);
  if (!rc) rc = launch_prune_compact(D->stream, d_raw, d_units, d_off, d_bcnt, W - 1, N - 1, (uint32_t)cap_units);
  if (!rc && (hipEventRecord(ev[1], D->stream) != hipSuccess ||
              hipMemcpyAsync(&pc, d_pc, sizeof pc, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
              hipMemcpyAsync(bcnt, d_bcnt, sizeof bcnt, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
              hipStreamSynchronize(D->stream) != hipSuccess))
    rc = BDEG_E_DEVICE;
  if (!rc && pc.overflow) rc = BDEG_E_STATE; // cannot happen: every bucket holds all its units
  pc.units = 0;
  for (int c = W - 1; c < N; c++) pc.units += bcnt[c];
  if (!rc) {
    LaunchShape shape = job.shape;
    shape.single = single_group(N);
    shape.dense = (job.sys[0].flags & SYS_DENSE) != 0;
    shape.mode = MODE_PLAIN;
    rc = launch_enumerate(D->stream, job.d_sys, job.d_pts, job.d_hts, d_units, pc.units, job.d_acc, job.d_cnt, k, k,
                          shape);
  }
  if (!rc && hipEventRecord(ev[2], D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
  std::vector<SysAcc> acc;
  if (!rc) rc = job_collect(job, D->stream, acc, nullptr);
  if (!rc) {
    *nvol = bdeg_u128{acc[0].lo, acc[0].hi};
    *tie = (int32_t)acc[0].tie;
    if (cells) *cells = acc[0].cells;
    if (ps) {
      float f = 0.f, g = 0.f;
      (void)hipEventElapsedTime(&f, ev[0], ev[1]);
      (void)hipEventElapsedTime(&g, ev[1], ev[2]);
      ps->prefixes = items.size();
      ps->degenerate = pc.degenerate;
      ps->pruned = pc.pruned;
      ps->units = pc.units;
      ps->pivots = pc.pivots;
      ps->prefix_size = d;
      ps->width = W;
      ps->filter_ms = f;
      ps->enum_ms = g;
    }
  }
  cleanup();
  return rc;
}


} // namespace bdeg

int bdeg_nvol_points_pruned(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, int32_t width,
                            bdeg_u128 *nvol, int32_t *tie, uint64_t *cells, bdeg_prune_stats *ps) {
  if (!nvol || !tie) return BDEG_E_ARG;
  int rc = check_points(points, heights, N, k);
  if (rc) return rc;
  PrunePlan P;
  if ((rc = prune_plan(N, k, width, P))) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  return prune_run(D, P, points, heights, N, k, nvol, tie, cells, ps);
}

int bdeg_cells_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t rank_lo,
                      uint64_t rank_hi, uint64_t cap, uint64_t *cell_masks, int64_t *normal_num,
                      uint64_t *normal_den, uint64_t *n_cells, int32_t *tie) {
  if (!n_cells || !tie || (cap > 0 && (!cell_masks || !normal_num || !normal_den))) return BDEG_E_ARG;
  int rc = check_points(points, heights, N, k);
  if (rc) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  Job job;
  points_job(job, points, heights, N, k, rank_lo, rank_hi);
  rc = job_upload(job);
  if (rc) return rc;
  SysAcc acc;
  rc = list_cells(D, job, N, k, cap, cell_masks, normal_num, normal_den, n_cells, &acc);
  if (rc) return rc;
  *tie = (int32_t)acc.tie;
  return BDEG_OK;
}

int bdeg_subdivision(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits, uint64_t cap,
                     int32_t *points, int64_t *heights, uint64_t *cell_masks, int64_t *normal_num,
                     uint64_t *normal_den, uint64_t *n_cells, bdeg_result *out) {
  if (!A || !out || !n_cells || !points || !heights || (cap > 0 && (!cell_masks || !normal_num || !normal_den)))
    return BDEG_E_ARG;
  *n_cells = 0;
  bdeg_result res;
  HostSys hs;
  if (!prepare_one(A, m, n, seed, lift_bits, 0, res, hs)) {
    *out = res;
    return res.status;
  }
  int st;
  Device *D = device_get(&st);
  if (!D) {
    res.status = st;
    *out = res;
    return st;
  }
  std::lock_guard<std::mutex> lk(D->mu);
  Job job;
  const uint64_t cand = binom_u64(hs.N, hs.k + 1);
  for (;;) {
    std::vector<HostSys> one{hs};
    job_build_seeded(job, one, choose_max_cost(cand, default_waves(hs.k, hs.k, 4)));
    int rc = job_upload(job);
    SysAcc acc{};
    uint64_t count = 0;
    if (!rc) rc = list_cells(D, job, hs.N, hs.k, cap, cell_masks, normal_num, normal_den, &count, &acc);
    if (!rc && hipMemcpyAsync(heights, job.d_hts, (size_t)hs.N * sizeof(int64_t), hipMemcpyDeviceToHost,
                              D->stream) != hipSuccess)
      rc = BDEG_E_DEVICE;
    if (!rc && hipStreamSynchronize(D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
    if (rc) {
      res.status = rc;
      break;
    }
    res.attempts = (int32_t)hs.attempt + 1;
    if (acc.tie) {
      if (hs.attempt + 1 >= BDEG_MAX_ATTEMPTS) {
        res.status = BDEG_E_TIE;
        break;
      }
      hs.attempt++;
      continue;
    }
    res.nvol = bdeg_u128{acc.lo, acc.hi};
    res.cells = acc.cells;
    res.status = BDEG_OK;
    *n_cells = count;
    memcpy(points, hs.pts.data(), hs.pts.size() * sizeof(int32_t));
    break;
  }
  *out = res;
  return res.status;
}

int bdeg_plan_units(int32_t N, int32_t k, uint64_t rank_lo, uint64_t rank_hi, uint64_t max_cost,
                    uint64_t *intervals, size_t cap, size_t *n_units) {
  if (!n_units || k < 1 || k > BDEG_MAX_K || N < k + 1 || N > 64 || max_cost == 0) return BDEG_E_ARG;
  std::vector<TileC> tc;
  tiles_range(N, k, 0, rank_lo, rank_hi, max_cost, tc);
  std::vector<Tile> tiles;
  tiles_sorted(tc, tiles);
  *n_units = tiles.size();
  if (tiles.size() > cap) return BDEG_E_NOMEM;
  for (size_t u = 0; u < tiles.size(); u++) tile_interval(tiles[u], k, &intervals[2 * u], &intervals[2 * u + 1]);
  return BDEG_OK;
}

} // extern "C"
