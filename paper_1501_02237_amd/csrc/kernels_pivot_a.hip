// Cell-walk kernels for k = 1..8, and the dispatch of all depths.
#include "pivot_device.hpp"

BDEG_PIVOT_INSTANCE(1)
BDEG_PIVOT_INSTANCE(2)
BDEG_PIVOT_INSTANCE(3)
BDEG_PIVOT_INSTANCE(4)
BDEG_PIVOT_INSTANCE(5)
BDEG_PIVOT_INSTANCE(6)
BDEG_PIVOT_INSTANCE(7)
BDEG_PIVOT_INSTANCE(8)

namespace bdeg {

#define BDEG_PIVOT_DECL(KK) PivotFn pivot_fn_##KK();
BDEG_PIVOT_DECL(9) BDEG_PIVOT_DECL(10) BDEG_PIVOT_DECL(11) BDEG_PIVOT_DECL(12) BDEG_PIVOT_DECL(13)
BDEG_PIVOT_DECL(14) BDEG_PIVOT_DECL(15) BDEG_PIVOT_DECL(16) BDEG_PIVOT_DECL(17) BDEG_PIVOT_DECL(18)
BDEG_PIVOT_DECL(19) BDEG_PIVOT_DECL(20) BDEG_PIVOT_DECL(21) BDEG_PIVOT_DECL(22) BDEG_PIVOT_DECL(23)
BDEG_PIVOT_DECL(24)
#undef BDEG_PIVOT_DECL

static PivotFn pivot_fn(int k) {
  switch (k) {
#define BDEG_PIVOT_CASE(KK) \
  case KK:                  \
    return pivot_fn_##KK();
    BDEG_PIVOT_CASE(1) BDEG_PIVOT_CASE(2) BDEG_PIVOT_CASE(3) BDEG_PIVOT_CASE(4) BDEG_PIVOT_CASE(5)
    BDEG_PIVOT_CASE(6) BDEG_PIVOT_CASE(7) BDEG_PIVOT_CASE(8) BDEG_PIVOT_CASE(9) BDEG_PIVOT_CASE(10)
    BDEG_PIVOT_CASE(11) BDEG_PIVOT_CASE(12) BDEG_PIVOT_CASE(13) BDEG_PIVOT_CASE(14) BDEG_PIVOT_CASE(15)
    BDEG_PIVOT_CASE(16) BDEG_PIVOT_CASE(17) BDEG_PIVOT_CASE(18) BDEG_PIVOT_CASE(19) BDEG_PIVOT_CASE(20)
    BDEG_PIVOT_CASE(21) BDEG_PIVOT_CASE(22) BDEG_PIVOT_CASE(23) BDEG_PIVOT_CASE(24)
#undef BDEG_PIVOT_CASE
    default:
      return nullptr;
  }
}

int max_pivot_blocks(int k) {
  PivotFn f = pivot_fn(k);
  if (!f) return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)f, 256, 0) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

int launch_pivot(void *stream, const PivotArgs &a, int k, int blocks) {
  PivotFn f = pivot_fn(k);
  if (!f || blocks <= 0) return BDEG_E_ARG;
  if (a.count == 0) return BDEG_OK;
  const uint64_t need = ((uint64_t)a.count + 3) / 4;
  if ((uint64_t)blocks > need) blocks = (int)need;
  hipLaunchKernelGGL(f, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

namespace dev {
// Rebuild the hash set after it has grown: one thread per slot of the old
// set (every cell, including those reached by pivots that never enter the list).
__global__ void __launch_bounds__(256) pivot_rehash_kernel(PivotArgs a, const uint64_t *old, uint64_t n_old) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i < n_old && old[i]) (void)set_insert(a, old[i]);
}
} // namespace dev

int launch_pivot_rehash(void *stream, const PivotArgs &a, const uint64_t *old, uint64_t n_old) {
  if (n_old == 0) return BDEG_OK;
  const uint64_t blocks = (n_old + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return BDEG_E_ARG;
  hipLaunchKernelGGL(dev::pivot_rehash_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a, old,
                     n_old);
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

} // namespace bdeg
