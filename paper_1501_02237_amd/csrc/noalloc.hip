// bdeg_nvol_points for callers that cannot allocate device memory (code
// under stream capture, tight serving loops, harnesses that forbid
// hipMalloc): the same work, volume and tie test (Section 4, eqs.
// "lower-face" and "simplex-vol"), with every device buffer the enumeration
// needs carved from one file-scope device array instead of hipMalloc'd
// memory.
//
// The array holds, at 256-byte aligned offsets: the system descriptor, its
// accumulator, the counter blocks of every launch range, the staged points
// and heights, and the work units.  Each GPU holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "api_internal.hpp"

namespace bdeg {
namespace noalloc {

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t OFF_SYS = 0;
constexpr size_t OFF_ACC = align256(OFF_SYS + sizeof(SysDesc));
constexpr size_t OFF_CNT = align256(OFF_ACC + sizeof(SysAcc));
constexpr size_t OFF_PTS = align256(OFF_CNT + (size_t)CNT_BLOCKS * sizeof(DevCounters));
constexpr size_t OFF_HTS = align256(OFF_PTS + (size_t)64 * BDEG_MAX_K * sizeof(int32_t));
constexpr size_t OFF_TILES = align256(OFF_HTS + (size_t)64 * sizeof(int64_t));
constexpr size_t BYTES = OFF_TILES + (size_t)BDEG_NOALLOC_MAX_UNITS * sizeof(Tile);
static_assert(BYTES <= BDEG_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds the published size");

} // namespace noalloc
} // namespace bdeg

static __device__ __align__(256) unsigned char scratch[BDEG_NOALLOC_SCRATCH_BYTES];

namespace bdeg {
namespace noalloc {

constexpr int MAX_DEVICES = 64;
static std::mutex g_mu;
static unsigned char *g_ptr[MAX_DEVICES]; // the array's device address on each GPU (nullptr: not set up)

// Device address of `scratch` on device `dev`, which must be current; looked
// up once per device.
static unsigned char *scratch_on(int dev, int *status) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev < 0 || dev >= MAX_DEVICES) {
    *status = BDEG_E_DEVICE;
    return nullptr;
  }
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      *status = BDEG_E_DEVICE;
      return nullptr;
    }
    g_ptr[dev] = (unsigned char *)p;
  }
  *status = BDEG_OK;
  return g_ptr[dev];
}

// The job's device pointers point into the scratch array for the duration of
// one call; they are cleared on every exit so that the job never frees them.
struct Borrow {
  Job &job;
  Borrow(Job &j, unsigned char *base) : job(j) {
    job.d_sys = (SysDesc *)(base + OFF_SYS);
    job.d_acc = (SysAcc *)(base + OFF_ACC);
    job.d_cnt = (DevCounters *)(base + OFF_CNT);
    job.d_pts = (int32_t *)(base + OFF_PTS);
    job.d_hts = (int64_t *)(base + OFF_HTS);
    job.d_tiles = (Tile *)(base + OFF_TILES);
    job.d_rerun = nullptr;
  }
  ~Borrow() {
    job.d_sys = nullptr;
    job.d_acc = nullptr;
    job.d_cnt = nullptr;
    job.d_pts = nullptr;
    job.d_hts = nullptr;
    job.d_tiles = nullptr;
    job.d_rerun = nullptr;
  }
};

} // namespace noalloc
} // namespace bdeg

using namespace bdeg;

extern "C" int bdeg_nvol_points_noalloc(const int32_t *points, const int64_t *heights, int32_t N, int32_t k,
                                        uint64_t rank_lo, uint64_t rank_hi, bdeg_u128 *nvol, int32_t *tie,
                                        uint64_t *cells) {
  if (!nvol || !tie) return BDEG_E_ARG;
  int rc = check_points(points, heights, N, k);
  if (rc) return rc;
  const uint64_t total = binom_u64(N, k + 1);
  const uint64_t hi = std::min(rank_hi, total), lo = std::min(rank_lo, hi);
  // even units of the largest size would not fit the array
  if ((hi - lo) / MAX_UNIT_CANDIDATES >= (uint64_t)BDEG_NOALLOC_MAX_UNITS) return BDEG_E_TOO_LARGE;
  int st;
  Device *D = device_get(&st); // makes the library's device current
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  unsigned char *base = noalloc::scratch_on(D->dev, &st);
  if (!base) return st;
  // host side of the plan, reused across calls (its device pointers are
  // borrowed from the scratch array below, never allocated)
  static Job job;
  uint64_t cost = 0; // 0: the default unit size; doubled while the plan has too many units
  for (;;) {
    points_job(job, points, heights, N, k, lo, hi, cost);
    if (job.tiles.size() <= (size_t)BDEG_NOALLOC_MAX_UNITS) break;
    cost = 2 * (cost ? cost : choose_max_cost(hi - lo, default_waves(k, k, 4)));
    if (cost > MAX_UNIT_CANDIDATES) return BDEG_E_TOO_LARGE;
  }
  noalloc::Borrow use(job, base);
  hipStream_t s = D->stream;
  if (hipMemcpyAsync(job.d_sys, job.sys.data(), sizeof(SysDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(job.d_pts, job.pts.data(), job.pts.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(job.d_hts, job.heights.data(), job.heights.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      (!job.tiles.empty() && hipMemcpyAsync(job.d_tiles, job.tiles.data(), job.tiles.size() * sizeof(Tile),
                                            hipMemcpyHostToDevice, s) != hipSuccess))
    return BDEG_E_DEVICE;
  // the clear kernel zeroes the accumulator and every counter block (the
  // array keeps the previous call's contents); then the enumeration
  rc = job_launch(job, s);
  if (rc) return rc;
  static std::vector<SysAcc> acc; // host readback, reused across calls
  rc = job_collect(job, s, acc, nullptr);
  if (rc) return rc;
  *nvol = bdeg_u128{acc[0].lo, acc[0].hi};
  *tie = (int32_t)acc[0].tie;
  if (cells) *cells = acc[0].cells;
  return BDEG_OK;
}
