// Device code of the cell walk (simplicial pivoting, paper Section 4.2-4.4):
// the regular subdivision is explored cell by cell across facets instead of
// deciding every (k+1)-subset, so the work follows the number of cells.
//
// One wavefront processes one cell C = {v_0 < ... } (a lower facet of the
// lifted points); lane j holds point j (N <= 64).
//   * Lane j's column is (a_j - a_{v0}, w_j - w_{v0}).  Fraction-free
//     Gauss-Jordan elimination with the k columns of C's other points as
//     pivots (row t is pivoted at step t, the pivot column is any unused cell
//     point with a nonzero entry there) turns column j into
//         (D lambda_1(j), ..., D lambda_k(j), D s_j),
//     where lambda are j's barycentric coordinates in the simplex C
//     (coordinate t belongs to the cell point pivoted at step t), s_j is the
//     height of lifted point j above C's hyperplane and D = det of C's edge
//     vectors (the last pivot; |D| is the cell's normalized volume).  Every
//     entry is a minor of the point matrix, so the device's certified widths
//     hold (spatial minors in int32, height minors in int64 split as
//     H1 2^31 + H0) and every division is exact.
//   * The neighbour of C across the facet opposite cell point v is
//     C - {v} + {u}, u minimizing s_u / (-lambda_v(u)) over the points with
//     lambda_v(u) < 0 (beyond the facet): the lifted hyperplane turning about
//     the facet meets u first (the simplicial pivot).  No such point: the
//     facet lies on the boundary of the convex hull.
//   * New cells enter a device hash set of vertex masks (one CAS per probe);
//     the first insertion appends the cell to the work list, so every cell is
//     processed exactly once and adds |D| to the volume.
// A point on C's hyperplane, or two points with the same minimal ratio, means
// the lifting is not generic: the walk reports a tie and the host redraws it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"
#include "exact_div.hpp"
#include "wave_ratio.hpp"

namespace bdeg {
namespace dev {

constexpr uint32_t PIVOT_LOW31 = 0x7FFFFFFFu;
constexpr int PIVOT_MAX_PROBE = 4096;


__device__ __forceinline__ int32_t prl(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int32_t pbp(int32_t v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
__device__ __forceinline__ uint64_t pballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint64_t cell_hash(uint64_t m) {
  m ^= m >> 33;
  m *= 0xFF51AFD7ED558CCDull;
  m ^= m >> 33;
  m *= 0xC4CEB9FE1A85EC53ull;
  m ^= m >> 33;
  return m;
}

// Insert a cell into the hash set; true when it was not there before.  Sets
// PIVOT_ERR_FULL when the probe sequence runs out.
__device__ __forceinline__ bool set_insert(const PivotArgs &a, uint64_t m) {
  uint64_t h = cell_hash(m) & a.table_mask;
  for (int p = 0; p < PIVOT_MAX_PROBE; p++) {
    const unsigned long long old = atomicCAS((unsigned long long *)&a.table[h], 0ull, (unsigned long long)m);
    if (old == 0ull) return true;
    if (old == m) return false;
    h = (h + 1) & a.table_mask;
  }
  atomicOr(&a.cnt->flags, PIVOT_ERR_FULL);
  return false;
}

template <int K>
__global__ void __launch_bounds__(256) pivot_kernel(PivotArgs a) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t vol = 0, cells = 0; // this wave's cells (uniform across the wave)
  for (;;) {
    // Every lane takes part in the claim (lane 0 adds one, the others zero)
    // and lane 0's result is read by index.  A claim made under a lane-0 branch
    // leaves a lane-dependent value at the loop header; the compiler may then
    // split the loop so that lanes 1..63 reach the broadcast without lane 0
    // and never leave it.
    const uint32_t claim = atomicAdd(&a.cnt->next, lane == 0 ? 1u : 0u);
    const uint32_t item = (uint32_t)__builtin_amdgcn_readlane((int32_t)claim, 0);
    if (item >= a.count) break;
    const uint64_t C = a.list[a.first + item];
    const int v0 = __builtin_ctzll(C);
    const bool valid = lane < a.N;
    // lane j's column: spatial differences and the split height difference
    int32_t x[K];
    int32_t H1 = 0, H0 = 0;
    if (valid) {
#pragma unroll
      for (int r = 0; r < K; r++) x[r] = a.pts[lane * K + r] - a.pts[v0 * K + r];
      const int64_t y = a.hts[lane] - a.hts[v0];
      H1 = (int32_t)(y >> 31);
      H0 = (int32_t)((uint32_t)y & PIVOT_LOW31);
    } else {
#pragma unroll
      for (int r = 0; r < K; r++) x[r] = 0;
    }
    uint64_t unused = C & ~(1ull << v0);
    int pivlane[K];
    int32_t prev = 1;
    bool singular = false;
#pragma unroll
    for (int t = 0; t < K; t++) {
      const uint64_t cand = pballot(((unused >> lane) & 1) && x[t] != 0) & unused;
      singular |= cand == 0;
      const int pl = cand ? __builtin_ctzll(cand) : v0; // (a singular cell is discarded below)
      pivlane[t] = pl;
      unused &= ~(1ull << pl);
      int32_t pc[K];
#pragma unroll
      for (int r = 0; r < K; r++) pc[r] = prl(x[r], pl);
      const int32_t ph1 = prl(H1, pl), ph0 = prl(H0, pl);
      const int32_t p = cand ? pc[t] : 1;
      const Div dv = make_div(prev);
      const int32_t xt = x[t];
#pragma unroll
      for (int r = 0; r < K; r++)
        if (r != t) x[r] = exdiv32((int64_t)p * x[r] - (int64_t)pc[r] * xt, dv);
      const int64_t A = (int64_t)p * H1 - (int64_t)ph1 * xt;
      const int64_t B = (int64_t)p * H0 - (int64_t)ph0 * xt;
      const int64_t h = exdiv_split(A, B, dv);
      H1 = (int32_t)(h >> 31);
      H0 = (int32_t)((uint32_t)h & PIVOT_LOW31);
      prev = p;
    }
    if (singular) { // a listed cell must be a full simplex
      if (lane == 0) atomicOr(&a.cnt->flags, PIVOT_ERR_STATE);
      continue;
    }
    // the cell, then a chain of neighbours: each one is reached by one pivot
    // of the tableau instead of a new elimination
    int32_t D = prev;
    uint64_t Cc = C;
    for (int hop = 0;; hop++) {
      const bool neg = D < 0;
      const bool in_c = (Cc >> lane) & 1;
      // height above the cell's hyperplane, times |D|
      const int64_t s_raw = (int64_t)H1 * ((int64_t)1 << 31) + (int64_t)(uint32_t)H0;
      const int64_t S = neg ? -s_raw : s_raw;
      const bool other = valid && !in_c;
      const uint64_t below = pballot(other && S < 0), on = pballot(other && S == 0);
      if (below) { // not a lower facet: the start cell was wrong, or a bug
        if (lane == 0) atomicOr(&a.cnt->flags, PIVOT_ERR_STATE);
        break;
      }
      if (on && lane == 0) atomicOr(&a.cnt->flags, PIVOT_TIE);
      vol += (uint64_t)(neg ? -(int64_t)D : (int64_t)D);
      cells++;
      // barycentric coordinate of the base point, times D
      int64_t sum = 0;
#pragma unroll
      for (int t = 0; t < K; t++) sum += x[t];
      const int64_t c0 = (int64_t)D - sum;
      // facets: opposite the point pivoted at step t (row t), then opposite v0;
      // lane t keeps the neighbour across facet t
      uint64_t mine = 0;
#pragma unroll
      for (int t = 0; t <= K; t++) {
        const int64_t c = t < K ? (int64_t)x[t] : c0;
        const int64_t cs = neg ? -c : c; // lambda * |D|
        const bool beyond = other && cs < 0;
        const RatioMin rm = ratio_min(beyond ? S : 0, beyond ? (int32_t)(-cs) : 0);
        const int u = rm.lane;
        if ((rm.lanes & (rm.lanes - 1)) && lane == 0) atomicOr(&a.cnt->flags, PIVOT_TIE); // equal minima
        if (u >= 0) { // (none: the facet is on the boundary of the hull)
          const int v = t < K ? pivlane[t] : v0;
          if (lane == t) mine = (Cc & ~(1ull << v)) | (1ull << u);
        }
      }
      // lane t inserts the neighbour across facet t: all probes in one round
      const bool fresh = mine && set_insert(a, mine);
      // the chain goes on into the first new neighbour across a facet t < k
      // (same base point) while the level's room allows
      const uint64_t fr = pballot(fresh) & ((1ull << K) - 1);
      int tc = -1;
      if (fr && hop < PIVOT_CHAIN_STEPS) { // (longer chains serialise a level)
        const uint32_t claim = atomicAdd(&a.cnt->chained, lane == 0 ? 1u : 0u);
        if ((uint32_t)prl((int32_t)claim, 0) < a.chain_budget) tc = __builtin_ctzll(fr);
      }
      if (fresh && lane != tc) {
        const uint32_t pos = atomicAdd(&a.cnt->tail, 1u);
        if (pos < a.cap_list)
          a.list[pos] = mine;
        else
          atomicOr(&a.cnt->flags, PIVOT_ERR_FULL);
      }
      if (tc < 0) break;
      // pivot: the point of row tc leaves, u enters; with e = x_tc(u),
      // x_r <- (e x_r - x_r(u) x_tc) / D for r != tc, row tc stays, D <- e
      const uint64_t nb = ((uint64_t)(uint32_t)prl((int32_t)(mine >> 32), tc) << 32) |
                          (uint32_t)prl((int32_t)(uint32_t)mine, tc);
      const int u = __builtin_ctzll(nb & ~Cc);
      int32_t pc[K];
#pragma unroll
      for (int r = 0; r < K; r++) pc[r] = prl(x[r], u);
      const int32_t ph1 = prl(H1, u), ph0 = prl(H0, u);
      int32_t e = 1, xt = 0;
#pragma unroll
      for (int r = 0; r < K; r++)
        if (r == tc) {
          e = pc[r];
          xt = x[r];
        }
      const Div dv = make_div(D);
#pragma unroll
      for (int r = 0; r < K; r++)
        if (r != tc) x[r] = exdiv32((int64_t)e * x[r] - (int64_t)pc[r] * xt, dv);
      const int64_t A = (int64_t)e * H1 - (int64_t)ph1 * xt;
      const int64_t B = (int64_t)e * H0 - (int64_t)ph0 * xt;
      const int64_t h = exdiv_split(A, B, dv);
      H1 = (int32_t)(h >> 31);
      H0 = (int32_t)((uint32_t)h & PIVOT_LOW31);
#pragma unroll
      for (int r = 0; r < K; r++)
        if (r == tc) pivlane[r] = u;
      D = e;
      Cc = nb;
    }
  }
  // the wave's tallies (uniform values) in one update
  if (lane == 0 && cells) {
    const unsigned long long old = atomicAdd(&a.cnt->vol_lo, (unsigned long long)vol);
    if (old + vol < old) atomicAdd(&a.cnt->vol_hi, 1ull);
    atomicAdd(&a.cnt->cells, (unsigned long long)cells);
  }
}

} // namespace dev
} // namespace bdeg

// Instantiation helper: bdeg::pivot_fn_<k>() for one k per line.
#define BDEG_PIVOT_INSTANCE(KK)                                                      \
  namespace bdeg {                                                                   \
  PivotFn pivot_fn_##KK() { return dev::pivot_kernel<KK>; }                          \
  }
