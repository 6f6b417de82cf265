// Extend (paper Section 4.1, the LP of eq. "ext-lp"; Section 4.5, Extend): a
// lower facet of a caller's lifting, found exactly, as the start cell of the
// walk.
//
// The paper grows a lower face one point at a time, deciding by a linear
// program whether the face plus a candidate point is still a lower face.
// Here each growth step is one exact supporting-hyperplane rotation, which
// answers the same question for the point it picks without a general LP:
//   * Start: the lowest lifted point b (smallest height, then smallest index)
//     is a lower vertex, supported by the horizontal hyperplane.
//   * State: F, a lower face, and for every point q its fraction-free residual
//     after eliminating F's points (Bareiss steps on the difference rows
//     a_q - a_b and heights w_q - w_b).  The spatial residual s_q holds q's
//     coordinates modulo the affine hull of F; the height residual h_q equals
//     c * v_q, where v_q is the value at q of a supporting functional of F
//     (zero on F, positive elsewhere) and c a known nonzero scale.
//   * Rotation: pick a live spatial column i and the sign sigma such that some
//     point has sigma * s_q[i] > 0; tilting the functional by t * sigma * e_i
//     lowers exactly those points, and the first one to reach zero, the
//     argmin of v_q / (sigma * s_q[i]) (compared exactly in 128-bit
//     products), joins F.  One Bareiss step on (that point, column i) makes
//     the new residual heights the tilted functional's values again, with
//     scale c * pivot / previous pivot.
//   * A point whose value is already zero lies on the face: it joins F by a
//     Bareiss step on any nonzero column of its spatial residual, and if that
//     residual is zero the face is not a simplex: the lifting is not generic
//     (a tie, as in the enumeration).
// After k eliminations F has k + 1 points with every other point strictly
// above its hyperplane: a lower facet.  Every residual is a bordered minor of
// the point matrix [1 | a | w], so the host's width certificate bounds them
// (spatial below 2^31, heights below 2^60) and each exact division is checked
// by multiplying back.  One wavefront, lane q = point q; the argmin and the
// column choice are scans by lane 0 over the shared residual table.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"
#include "exact_div.hpp"

namespace bdeg {
namespace dev {

__global__ void __launch_bounds__(64) extend_kernel(const int32_t *__restrict__ pts, const int64_t *__restrict__ hts,
                                                    int N, int K, ExtendResult *__restrict__ out) {
  __shared__ int32_t S[64][PIVOT_MAX_K]; // spatial residuals, all K columns kept in place
  __shared__ int64_t H[64];              // height residuals
  __shared__ int32_t prow[PIVOT_MAX_K];  // the pivot point's row, read before the update
  __shared__ int64_t ph;
  __shared__ int sh_p, sh_col, sh_state; // pivot point, pivot column, 0 running / 1 done / 2 tie / 3 error
  const int q = threadIdx.x;
  const bool valid = q < N;
  if (q == 0) {
    int b = 0;
    for (int j = 1; j < N; j++)
      if (hts[j] < hts[b]) b = j;
    sh_p = b;
    sh_state = 0;
  }
  __syncthreads();
  const int b = sh_p;
  for (int i = 0; i < K; i++) S[q][i] = valid ? pts[q * K + i] - pts[b * K + i] : 0;
  H[q] = valid ? hts[q] - hts[b] : 0;
  uint64_t F = 1ull << b;         // the face's points (uniform)
  uint64_t live = (1ull << K) - 1; // spatial columns not yet eliminated (uniform)
  int32_t prev = 1;
  int csign = 1; // sign of the scale c of the height residuals
  uint32_t bad = 0;
  const uint64_t points = N >= 64 ? ~0ull : ((1ull << N) - 1);
  __syncthreads();
  while (live) {
    if (q == 0) {
      sh_p = -1;
      sh_col = -1;
      // a point already on the face's hyperplane joins first (no rotation)
      for (int j = 0; j < N && sh_p < 0; j++) {
        if ((F >> j) & 1 || H[j] != 0) continue;
        for (int i = 0; i < K && sh_col < 0; i++)
          if ((live >> i) & 1 && S[j][i] != 0) sh_col = i;
        if (sh_col < 0) sh_state = 2; // affinely dependent on a lower face: not generic
        sh_p = j;
      }
      if (sh_p < 0) {
        // rotate about F: the first live column in which some point leaves aff(F)
        for (int i = 0; i < K && sh_col < 0; i++) {
          if (!((live >> i) & 1)) continue;
          for (int j = 0; j < N; j++)
            if (!((F >> j) & 1) && S[j][i] != 0) {
              sh_col = i;
              break;
            }
        }
        if (sh_col < 0) {
          sh_state = 3; // the points do not span the space
        } else {
          const int i = sh_col;
          int sigma = -1;
          for (int j = 0; j < N; j++)
            if (!((F >> j) & 1) && S[j][i] > 0) sigma = 1;
          // argmin of (csign * H[j]) / (sigma * S[j][i]) over sigma * S[j][i] > 0; the
          // numerators are positive (zero ones joined above)
          int best = -1;
          for (int j = 0; j < N; j++) {
            if ((F >> j) & 1) continue;
            const int64_t den = sigma > 0 ? (int64_t)S[j][i] : -(int64_t)S[j][i];
            if (den <= 0) continue;
            if (best < 0) {
              best = j;
              continue;
            }
            const int64_t dbest = sigma > 0 ? (int64_t)S[best][i] : -(int64_t)S[best][i];
            const __int128 lhs = (__int128)(csign * H[j]) * dbest, rhs = (__int128)(csign * H[best]) * den;
            if (lhs < rhs) best = j; // equal ratios: the others reach the hyperplane too and join next
          }
          sh_p = best;
        }
      }
      if (sh_p >= 0 && sh_col >= 0) {
        for (int i = 0; i < K; i++) prow[i] = S[sh_p][i];
        ph = H[sh_p];
      }
    }
    __syncthreads();
    if (sh_state != 0) break;
    const int p = sh_p, i = sh_col;
    const int32_t piv = prow[i];
    const int32_t sqi = S[q][i];
    const Div dv = make_div(prev);
    // one Bareiss step on (p, i) for every lane (F's rows and p's own become zero)
    for (int l = 0; l < K; l++) {
      if (!((live >> l) & 1) || l == i) continue;
      const int64_t v = (int64_t)piv * S[q][l] - (int64_t)prow[l] * sqi;
      const int32_t w = exdiv32(v, dv);
      bad |= (int64_t)w * prev != v;
      S[q][l] = w;
    }
    {
      const __int128 v = (__int128)piv * H[q] - (__int128)ph * sqi;
      const int64_t w = exdiv128(v, dv);
      bad |= (__int128)w * prev != v;
      H[q] = w;
    }
    S[q][i] = 0;
    csign = csign * (piv < 0 ? -1 : 1) * (prev < 0 ? -1 : 1);
    prev = piv;
    F |= 1ull << p;
    live &= ~(1ull << i);
    __syncthreads();
  }
  // every point off the facet must lie strictly above it
  const bool below_or_on = valid && !((F >> q) & 1) && csign * H[q] <= 0;
  const uint64_t m = __builtin_amdgcn_ballot_w64(below_or_on);
  const uint64_t anybad = __builtin_amdgcn_ballot_w64(bad != 0);
  if (q == 0) {
    uint32_t flags = 0;
    if (sh_state == 2 || (sh_state == 0 && m)) flags |= EXTEND_TIE;
    if (sh_state == 3) flags |= EXTEND_ERR_SPAN;
    if (anybad) flags |= EXTEND_ERR_RANGE;
    out->mask = (sh_state == 0) ? (F & points) : 0;
    out->flags = flags;
  }
}

} // namespace dev

int launch_extend(void *stream, const int32_t *d_pts, const int64_t *d_hts, int N, int k, ExtendResult *d_out) {
  if (k < 1 || k > PIVOT_MAX_K || N < k + 1 || N > 64 || !d_pts || !d_hts || !d_out) return BDEG_E_ARG;
  hipLaunchKernelGGL(dev::extend_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, d_pts, d_hts, N, k, d_out);
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

} // namespace bdeg
