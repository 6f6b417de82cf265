// Inner normals of the cells (lower facets) listed by the enumeration kernel.
//
// A cell with vertices c_0 < ... < c_k of the lifted points has a unique inner
// normal (alpha, 1) (Section 5, eq. "lower-d-face-again"): <a_v, alpha> + w_v
// takes the same value at every vertex v and a larger one at every other
// point.  With the rows x_j = (a_{c_j} - a_{c_0}, w_{c_j} - w_{c_0}),
// j = 1..k, of X = [M | dw] (M the k x k spatial block), alpha solves
// M alpha = -dw.  Its exact form is the null vector n of X with n_k = det M
// (the cofactor vector): alpha = n_{0..k-1} / n_k, listed as
// num = sign(n_k) n_{0..k-1} and den = |n_k|, the cell's normalized volume.
//
// One thread per cell (cells are few next to the candidates; this pass is a
// small fraction of the enumeration); unrolled per k up to 12, a runtime-k
// version above.  Fraction-free (Bareiss) elimination of X
// with row pivoting on the spatial columns leaves an upper-triangular U whose
// last pivot is det M up to the sign of the row permutation; taking
// n_k = U[k-1][k-1], back substitution
//     n_i = -(sum_{j>i} U[i][j] n_j + U[i][k] n_k) / U[i][i]
// divides exactly (n is an integer multiple of the cofactor vector, by +-1).
// Spatial entries are minors of the differences (certified below 2^31), the
// height column and the n_j stay below 2^60, so every product fits 96 bits;
// every division is checked by multiplying back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"
#include "exact_div.hpp"

namespace bdeg {
namespace dev {

constexpr uint32_t CELL_ERR_MASK = 1;  // a listed mask is not a (k+1)-subset of the points
constexpr uint32_t CELL_ERR_RANGE = 2; // D = 0 or a value outside the certified widths

template <int K>
__global__ void __launch_bounds__(256) cell_normals_kernel(const uint64_t *__restrict__ masks, uint64_t n,
                                                           const int32_t *__restrict__ pts,
                                                           const int64_t *__restrict__ hts, int N,
                                                           int64_t *__restrict__ num, uint64_t *__restrict__ den,
                                                           uint32_t *__restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t m = masks[i];
  const uint64_t allowed = N >= 64 ? ~0ull : ((1ull << N) - 1);
  if (__builtin_popcountll(m) != K + 1 || (m & ~allowed)) {
    atomicOr(err, CELL_ERR_MASK);
    return;
  }
  const int c0 = __builtin_ctzll(m);
  m &= m - 1;
  int32_t a[K][K]; // spatial block
  int64_t h[K];    // height column
#pragma unroll
  for (int r = 0; r < K; r++) {
    const int c = __builtin_ctzll(m);
    m &= m - 1;
#pragma unroll
    for (int q = 0; q < K; q++) a[r][q] = pts[c * K + q] - pts[c0 * K + q];
    h[r] = hts[c] - hts[c0];
  }
  bool bad = false;
  int32_t prev = 1;
#pragma unroll
  for (int t = 0; t < K; t++) {
    // the first row at or below t with a nonzero entry in column t becomes row t
#pragma unroll
    for (int r = t + 1; r < K; r++) {
      const bool sw = a[t][t] == 0 && a[r][t] != 0;
#pragma unroll
      for (int q = t; q < K; q++) {
        const int32_t x = a[t][q], y = a[r][q];
        a[t][q] = sw ? y : x;
        a[r][q] = sw ? x : y;
      }
      const int64_t x = h[t], y = h[r];
      h[t] = sw ? y : x;
      h[r] = sw ? x : y;
    }
    const int32_t piv = a[t][t];
    bad |= piv == 0;
    if (t + 1 < K) {
      const Div dv = make_div(prev);
#pragma unroll
      for (int r = t + 1; r < K; r++) {
        const int32_t art = a[r][t];
#pragma unroll
        for (int q = t + 1; q < K; q++) {
          const int64_t v = (int64_t)piv * a[r][q] - (int64_t)art * a[t][q];
          const int32_t w = exdiv32(v, dv);
          bad |= (int64_t)w * prev != v;
          a[r][q] = w;
        }
        const __int128 v = (__int128)piv * h[r] - (__int128)art * h[t];
        const int64_t w = exdiv128(v, dv);
        bad |= (__int128)w * prev != v;
        h[r] = w;
      }
    }
    prev = piv != 0 ? piv : 1;
  }
  int64_t nv[K + 1];
  nv[K] = a[K - 1][K - 1];
#pragma unroll
  for (int r = K - 1; r >= 0; r--) {
    __int128 s = (__int128)h[r] * nv[K];
#pragma unroll
    for (int j = r + 1; j < K; j++) s += (__int128)a[r][j] * nv[j];
    const int32_t d = a[r][r] != 0 ? a[r][r] : 1;
    const int64_t w = exdiv128(-s, make_div(d));
    bad |= (__int128)w * d != -s;
    nv[r] = w;
  }
  const int64_t nk = nv[K];
  const bool flip = nk < 0;
#pragma unroll
  for (int q = 0; q < K; q++) num[i * K + q] = flip ? -nv[q] : nv[q];
  den[i] = (uint64_t)(flip ? -nk : nk);
  if (bad) atomicOr(err, CELL_ERR_RANGE);
}

// The same for k > 12 with the dimension read at run time (loops instead of
// unrolled code; the matrix lives in private memory).  Cells of such systems
// are few next to their candidates, and unrolled instances this deep take
// minutes to compile.
constexpr int DEEP_K_MAX = PIVOT_MAX_K; // the walk's cells reach k = 24
__global__ void __launch_bounds__(256) cell_normals_deep_kernel(const uint64_t *__restrict__ masks, uint64_t n,
                                                                const int32_t *__restrict__ pts,
                                                                const int64_t *__restrict__ hts, int N, int K,
                                                                int64_t *__restrict__ num,
                                                                uint64_t *__restrict__ den,
                                                                uint32_t *__restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t m = masks[i];
  const uint64_t allowed = N >= 64 ? ~0ull : ((1ull << N) - 1);
  if (K < 1 || K > DEEP_K_MAX || __builtin_popcountll(m) != K + 1 || (m & ~allowed)) {
    atomicOr(err, CELL_ERR_MASK);
    return;
  }
  const int c0 = __builtin_ctzll(m);
  m &= m - 1;
  int32_t a[DEEP_K_MAX][DEEP_K_MAX];
  int64_t h[DEEP_K_MAX];
#pragma unroll 1
  for (int r = 0; r < K; r++) {
    const int c = __builtin_ctzll(m);
    m &= m - 1;
#pragma unroll 1
    for (int q = 0; q < K; q++) a[r][q] = pts[c * K + q] - pts[c0 * K + q];
    h[r] = hts[c] - hts[c0];
  }
  bool bad = false;
  int32_t prev = 1;
#pragma unroll 1
  for (int t = 0; t < K; t++) {
    int p = t;
    while (p < K && a[p][t] == 0) p++;
    if (p == K) {
      bad = true; // D = 0: not a cell
      break;
    }
    if (p != t) {
#pragma unroll 1
      for (int q = t; q < K; q++) {
        const int32_t x = a[t][q];
        a[t][q] = a[p][q];
        a[p][q] = x;
      }
      const int64_t x = h[t];
      h[t] = h[p];
      h[p] = x;
    }
    const int32_t piv = a[t][t];
    const Div dv = make_div(prev);
#pragma unroll 1
    for (int r = t + 1; r < K; r++) {
      const int32_t art = a[r][t];
#pragma unroll 1
      for (int q = t + 1; q < K; q++) {
        const int64_t v = (int64_t)piv * a[r][q] - (int64_t)art * a[t][q];
        const int32_t w = exdiv32(v, dv);
        bad |= (int64_t)w * prev != v;
        a[r][q] = w;
      }
      const __int128 v = (__int128)piv * h[r] - (__int128)art * h[t];
      const int64_t w = exdiv128(v, dv);
      bad |= (__int128)w * prev != v;
      h[r] = w;
    }
    prev = piv;
  }
  int64_t nv[DEEP_K_MAX + 1];
  if (!bad) {
    nv[K] = a[K - 1][K - 1];
#pragma unroll 1
    for (int r = K - 1; r >= 0; r--) {
      __int128 s = (__int128)h[r] * nv[K];
#pragma unroll 1
      for (int j = r + 1; j < K; j++) s += (__int128)a[r][j] * nv[j];
      const int32_t d = a[r][r];
      const int64_t w = exdiv128(-s, make_div(d));
      bad |= (__int128)w * d != -s;
      nv[r] = w;
    }
  }
  if (bad) {
    atomicOr(err, CELL_ERR_RANGE);
    return;
  }
  const int64_t nk = nv[K];
  const bool flip = nk < 0;
#pragma unroll 1
  for (int q = 0; q < K; q++) num[i * K + q] = flip ? -nv[q] : nv[q];
  den[i] = (uint64_t)(flip ? -nk : nk);
}

} // namespace dev

int launch_cell_normals(void *stream, const uint64_t *d_masks, uint64_t n, const int32_t *d_pts,
                        const int64_t *d_hts, int N, int k, int64_t *d_num, uint64_t *d_den, uint32_t *d_err) {
  if (n == 0) return BDEG_OK;
  if (k < 1 || k > PIVOT_MAX_K || N < k + 1 || N > 64 || !d_masks || !d_pts || !d_hts || !d_num || !d_den || !d_err)
    return BDEG_E_ARG;
  const uint64_t blocks = (n + 255) / 256;
  if (blocks > 0x7FFFFFFFull) return BDEG_E_TOO_LARGE;
  const dim3 grid((unsigned)blocks), block(256);
  hipStream_t s = (hipStream_t)stream;
  switch (k) {
#define BDEG_CELL_CASE(KK)                                                                                   \
  case KK:                                                                                                   \
    hipLaunchKernelGGL(dev::cell_normals_kernel<KK>, grid, block, 0, s, d_masks, n, d_pts, d_hts, N, d_num, \
                       d_den, d_err);                                                                        \
    break;
    BDEG_CELL_CASE(1) BDEG_CELL_CASE(2) BDEG_CELL_CASE(3) BDEG_CELL_CASE(4) BDEG_CELL_CASE(5) BDEG_CELL_CASE(6)
    BDEG_CELL_CASE(7) BDEG_CELL_CASE(8) BDEG_CELL_CASE(9) BDEG_CELL_CASE(10) BDEG_CELL_CASE(11)
    BDEG_CELL_CASE(12)
#undef BDEG_CELL_CASE
    default:
      hipLaunchKernelGGL(dev::cell_normals_deep_kernel, grid, block, 0, s, d_masks, n, d_pts, d_hts, N, k, d_num,
                         d_den, d_err);
      break;
  }
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

} // namespace bdeg
