// Small device kernels (lifting, clearing) and the launch helpers of the
// enumeration kernels, which are instantiated in kernels_k*.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"

namespace bdeg {
namespace dev {

// heights of the listed systems (all systems when active == nullptr)
__global__ void lift_kernel(const SysDesc *__restrict__ sys, const int32_t *__restrict__ active, int n_active,
                            int64_t *__restrict__ hts) {
  const int s = blockIdx.x;
  if (s >= n_active) return;
  const int sid = active ? active[s] : s;
  const SysDesc d = sys[sid];
  const int j = threadIdx.x;
  if (j < d.N) hts[d.ht_off + j] = lift_height(d.lift_key, j, d.lift_bits);
}

__device__ __forceinline__ void clear_acc(SysAcc *a, uint32_t attempt) {
  a->lo = 0;
  a->hi = 0;
  a->cells = 0;
  a->tie = 0;
  a->attempt = attempt;
}

__device__ __forceinline__ void clear_counters(DevCounters *cnt) {
  cnt->ridges = cnt->inner = cnt->sp_upd = cnt->pruned = cnt->leaves = cnt->tiles = 0;
  cnt->rsteps = cnt->lsteps = cnt->lempty = 0;
  cnt->w_inner = cnt->w_spatial = cnt->w_ridges = cnt->w_leaves = 0;
  cnt->triples = cnt->dunits = cnt->quads = 0;
  cnt->next_tile = 0;
  cnt->error = 0;
}

// every system back to attempt 0; counters and redraw gates cleared
__global__ void reset_kernel(SysDesc *__restrict__ sys, SysAcc *__restrict__ acc, int n_sys,
                             DevCounters *__restrict__ cnt, int n_cnt, uint32_t *__restrict__ rerun, int rounds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sys) {
    sys[i].lift_key = lift_key(sys[i].seed, sys[i].sys_index, 0);
    clear_acc(&acc[i], 0);
  }
  if (i < n_cnt) clear_counters(&cnt[i]);
  if (i < rounds) rerun[(size_t)i * (n_sys + 1)] = 0;
}

// one in-pass redraw round (one thread per system; a system's heights are
// rewritten by its own thread, at most 64 points)
__global__ void retie_kernel(SysDesc *__restrict__ sys, SysAcc *__restrict__ acc, int64_t *__restrict__ hts,
                             int n_sys, uint32_t *__restrict__ rerun) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  const SysAcc a = acc[s];
  uint32_t act = 0;
  if (a.tie && a.attempt + 1 < (uint32_t)BDEG_MAX_ATTEMPTS) {
    SysDesc &d = sys[s];
    const uint32_t att = a.attempt + 1;
    d.lift_key = lift_key(d.seed, d.sys_index, att);
    for (int j = 0; j < d.N; j++) hts[d.ht_off + j] = lift_height(d.lift_key, j, d.lift_bits);
    clear_acc(&acc[s], att);
    act = 1;
    atomicOr(&rerun[0], 1u);
  }
  rerun[1 + s] = act;
}

__global__ void clear_kernel(SysAcc *__restrict__ acc, int n_sys, DevCounters *__restrict__ cnt_all, int n_cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sys) clear_acc(&acc[i], 0);
  if (i < n_cnt && cnt_all) clear_counters(cnt_all + i);
}

// clear the partial sums of the listed systems
__global__ void clear_list_kernel(SysAcc *__restrict__ acc, const int32_t *__restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) clear_acc(&acc[list[i]], 0);
}

} // namespace dev

// ---------------------------------------------------------------- launch helpers
static int hip_ok(hipError_t e) { return e == hipSuccess ? BDEG_OK : BDEG_E_DEVICE; }

int launch_lift(void *stream, const SysDesc *d_sys, const int32_t *d_active, int n_active, int64_t *d_heights) {
  if (n_active <= 0) return BDEG_OK;
  hipLaunchKernelGGL(dev::lift_kernel, dim3(n_active), dim3(64), 0, (hipStream_t)stream, d_sys, d_active,
                     n_active, d_heights);
  return hip_ok(hipGetLastError());
}

int launch_clear(void *stream, SysAcc *d_acc, int n_sys, DevCounters *d_cnt, int n_cnt) {
  int n = n_sys > n_cnt ? n_sys : n_cnt;
  if (n < 1) n = 1;
  hipLaunchKernelGGL(dev::clear_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_acc, n_sys,
                     d_cnt, n_cnt);
  return hip_ok(hipGetLastError());
}

int launch_reset(void *stream, SysDesc *d_sys, SysAcc *d_acc, int n_sys, DevCounters *d_cnt, int n_cnt,
                 uint32_t *d_rerun, int rounds) {
  int n = n_sys > n_cnt ? n_sys : n_cnt;
  if (rounds > n) n = rounds;
  if (n < 1) n = 1;
  hipLaunchKernelGGL(dev::reset_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_sys, d_acc, n_sys,
                     d_cnt, n_cnt, d_rerun, rounds);
  return hip_ok(hipGetLastError());
}

int launch_retie(void *stream, SysDesc *d_sys, SysAcc *d_acc, int64_t *d_heights, int n_sys, uint32_t *d_rerun) {
  if (n_sys <= 0) return BDEG_OK;
  hipLaunchKernelGGL(dev::retie_kernel, dim3((n_sys + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_sys, d_acc,
                     d_heights, n_sys, d_rerun);
  return hip_ok(hipGetLastError());
}

int launch_clear_list(void *stream, SysAcc *d_acc, const int32_t *d_list, int n) {
  if (n <= 0) return BDEG_OK;
  hipLaunchKernelGGL(dev::clear_list_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_acc, d_list,
                     n);
  return hip_ok(hipGetLastError());
}

// per-k-range instantiations (kernels_k*.hip)
EnumFn enum_fn_1_1(int, int);
EnumFn enum_fn_2_2(int, int);
EnumFn enum_fn_3_3(int, int);
EnumFn enum_fn_4_4(int, int);
EnumFn enum_fn_5_5(int, int);
EnumFn enum_fn_6_6(int, int);
EnumFn enum_fn_7_7(int, int);
EnumFn enum_fn_8_8(int, int);
EnumFn enum_fn_9_9(int, int);
EnumFn enum_fn_10_10(int, int);
EnumFn enum_fn_11_11(int, int);
EnumFn enum_fn_12_12(int, int);
EnumFn enum_fn_13_13(int, int);
EnumFn enum_fn_14_14(int, int);
EnumFn enum_fn_15_15(int, int);
EnumFn enum_fn_16_16(int, int);
EnumFn enum_fn_17_17(int, int);
EnumFn enum_fn_18_18(int, int);
EnumFn enum_fn_1_7(int, int);
EnumFn enum_fn_1_12(int, int);

// Single-k kernels (exact register budget) and mixed-k kernels for batches,
// each in three variants: lane groups read per system (0), one point group
// per wavefront (1, N > 32), and the lane-dense kernel (2, k >= 3); `mode`
// selects plain, counting (MODE_STATS) or cell-listing (MODE_EMIT, single-k
// only).
static EnumFn enum_fn(int klo, int khi, int mode, int variant) {
  if (klo == khi) {
    switch (khi) {
      case 1: return enum_fn_1_1(mode, variant);
      case 2: return enum_fn_2_2(mode, variant);
      case 3: return enum_fn_3_3(mode, variant);
      case 4: return enum_fn_4_4(mode, variant);
      case 5: return enum_fn_5_5(mode, variant);
      case 6: return enum_fn_6_6(mode, variant);
      case 7: return enum_fn_7_7(mode, variant);
      case 8: return enum_fn_8_8(mode, variant);
      case 9: return enum_fn_9_9(mode, variant);
      case 10: return enum_fn_10_10(mode, variant);
      case 11: return enum_fn_11_11(mode, variant);
      case 12: return enum_fn_12_12(mode, variant);
      case 13: return enum_fn_13_13(mode, variant);
      case 14: return enum_fn_14_14(mode, variant);
      case 15: return enum_fn_15_15(mode, variant);
      case 16: return enum_fn_16_16(mode, variant);
      case 17: return enum_fn_17_17(mode, variant);
      case 18: return enum_fn_18_18(mode, variant);
      default: return nullptr;
    }
  }
  if (khi <= 7) return enum_fn_1_7(mode, variant);
  if (khi <= 12) return enum_fn_1_12(mode, variant);
  return nullptr;
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

static int variant_of(bool single, bool dense) { return dense ? 2 : single ? 1 : 0; }

int max_enum_blocks(int klo, int khi, int waves_per_block, bool single, bool dense) {
  EnumFn f = enum_fn(klo, khi, MODE_PLAIN, variant_of(single, dense));
  if (!f) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)f, waves_per_block * 64, 0) != hipSuccess)
    return 0;
  return per_cu * device_cu_count();
}

int launch_enumerate(void *stream, const SysDesc *d_sys, const int32_t *d_pts, const int64_t *d_heights,
                     const Tile *d_tiles, uint32_t n_tiles, SysAcc *d_acc, DevCounters *d_cnt, int klo, int khi,
                     LaunchShape shape) {
  EnumFn f = enum_fn(klo, khi, shape.mode, variant_of(shape.single, shape.dense));
  if (shape.mode == MODE_EMIT && (!shape.sink.count || (shape.sink.cap > 0 && !shape.sink.masks))) return BDEG_E_ARG;
  if (!f) return BDEG_E_TOO_LARGE;
  if (n_tiles == 0) return BDEG_OK;
  int blocks = shape.blocks;
  const int wpb = shape.waves_per_block > 0 ? shape.waves_per_block : 4;
  if (blocks <= 0) blocks = max_enum_blocks(klo, khi, wpb, shape.single, shape.dense);
  if (blocks <= 0) return BDEG_E_DEVICE;
  const uint64_t need = ((uint64_t)n_tiles + wpb - 1) / wpb;
  if ((uint64_t)blocks > need) blocks = (int)need;
  hipLaunchKernelGGL(f, dim3(blocks), dim3(wpb * 64), 0, (hipStream_t)stream, d_sys, d_pts, d_heights, d_tiles,
                     n_tiles, d_acc, d_cnt, shape.sink, shape.rerun);
  return hip_ok(hipGetLastError());
}

} // namespace bdeg
