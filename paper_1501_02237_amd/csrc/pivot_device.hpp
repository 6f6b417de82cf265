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
//     the first insertion claims the cell, so every cell is processed exactly
//     once and adds |D| to the volume.  A claimed cell is either reached at
//     once by a pivot of the tableau (depth first, left again by the inverse
//     pivot) or appended to the work list of the next level.
//   * A wave goes from one listed cell to the next by a pivot per point that
//     differs (consecutive entries are mostly siblings), moving the base
//     point when needed, and eliminates afresh only when that fails.
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

// (at least 5 waves per SIMD: at k = 20..24 that spills a few VGPRs, and the
// walk of k = 22 is faster for it than at 4 waves without spills)
template <int K>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) pivot_kernel(PivotArgs a) {
  const int lane = (int)(threadIdx.x & 63);
  const int wv = (int)(threadIdx.x >> 6);
  uint64_t vol = 0, cells = 0; // this wave's cells (uniform across the wave)
  uint32_t credit = 0;         // room the wave holds (uniform), in insertions
  // the depth-first pivots of each wave: per depth the rows reserved, the
  // point entering across each reserved row (lane = row), and how the cell
  // at that depth was entered (row and the point that left)
  __shared__ uint8_t s_u[4][PIVOT_DFS_MAX + 1][64];
  __shared__ uint32_t s_res[4][PIVOT_DFS_MAX + 1];
  __shared__ uint8_t s_row[4][PIVOT_DFS_MAX + 1], s_left[4][PIVOT_DFS_MAX + 1];
  // cells one claimed cell may reach by pivots: few while the level has
  // fewer cells than the grid has waves (long serial runs would hold the
  // level up), more as the level widens
  const uint32_t waves = gridDim.x * 4u;
  const bool wide = a.count >= 16u * waves;
  const uint32_t item_reach = wide ? (uint32_t)PIVOT_DFS_MAX : a.count >= 2u * waves ? 8u : 2u;
  // cells a wave claims at once (consecutive entries, so that the next one
  // is mostly a few pivots away), and its list appends collected in LDS:
  // the shared counters then take one atomic per several cells
  const uint32_t batch = wide ? (uint32_t)PIVOT_CLAIM_BATCH : 4u;
  __shared__ uint64_t s_buf[4][64];
  uint32_t nbuf = 0; // (uniform)
  const auto flush = [&]() {
    const uint32_t pos = (uint32_t)prl((int32_t)atomicAdd(&a.cnt->tail, lane == 0 ? nbuf : 0u), 0);
    if ((uint32_t)lane < nbuf) {
      if (pos + (uint32_t)lane < a.cap_list)
        a.list[pos + lane] = s_buf[wv][lane];
      else
        atomicOr(&a.cnt->flags, PIVOT_ERR_FULL);
    }
    nbuf = 0;
  };
  // the tableau (lane j = point j), kept from one claimed cell to the next
  const bool valid = lane < a.N;
  int32_t x[K];
  int32_t H1 = 0, H0 = 0;
  int pivlane[K]; // the point pivoted at step t (row t)
  int32_t D = 1;
  uint64_t Cc = 0;
  int v0 = 0;
  bool have = false; // the tableau holds the last claimed cell
  // pivot: the point of row tp leaves, point up enters; with e = x_tp(up),
  // x_r <- (e x_r - x_r(up) x_tp) / D for r != tp, row tp stays, D <- e.
  // Applied with the point that left, it restores the tableau before.
  // Returns the point that left.
  const auto pivot = [&](int tp, int up) {
    int32_t pc[K];
#pragma unroll
    for (int r = 0; r < K; r++) pc[r] = prl(x[r], up);
    const int32_t ph1 = prl(H1, up), ph0 = prl(H0, up);
    int32_t e = 1, xt = 0;
    int vout = 0;
#pragma unroll
    for (int r = 0; r < K; r++)
      if (r == tp) {
        e = pc[r];
        xt = x[r];
        vout = pivlane[r];
      }
    const Div dv = make_div(D);
#pragma unroll
    for (int r = 0; r < K; r++)
      if (r != tp) x[r] = exdiv32((int64_t)e * x[r] - (int64_t)pc[r] * xt, dv);
    const int64_t A = (int64_t)e * H1 - (int64_t)ph1 * xt;
    const int64_t B = (int64_t)e * H0 - (int64_t)ph0 * xt;
    const int64_t h = exdiv_split(A, B, dv);
    H1 = (int32_t)(h >> 31);
    H0 = (int32_t)((uint32_t)h & PIVOT_LOW31);
#pragma unroll
    for (int r = 0; r < K; r++)
      if (r == tp) pivlane[r] = up;
    D = e;
    Cc = (Cc & ~(1ull << vout)) | (1ull << up);
    return vout;
  };
  uint32_t next_item = 0, claimed = 0;
  for (;;) {
    // Every lane takes part in the claim (lane 0 adds, the others add zero)
    // and lane 0's result is read by index.  A claim made under a lane-0 branch
    // leaves a lane-dependent value at the loop header; the compiler may then
    // split the loop so that lanes 1..63 reach the broadcast without lane 0
    // and never leave it.
    if (claimed == 0) {
      const uint32_t claim = atomicAdd(&a.cnt->next, lane == 0 ? batch : 0u);
      next_item = (uint32_t)__builtin_amdgcn_readlane((int32_t)claim, 0);
      claimed = batch;
    }
    const uint32_t item = next_item++;
    claimed--;
    if (item >= a.count) break;
    const uint64_t C = a.list[a.first + item];
    // From the last claimed cell by pivots when both differ in a few points
    // (consecutive list entries are mostly siblings), else a new
    // elimination.  A pivot with a zero entry (no point of the new cell can
    // replace a leaving one in its row) falls back too.
    bool elim = true;
    if (have && __builtin_popcountll(Cc & ~C) <= PIVOT_SWAPS && (Cc & C)) {
      if (!((C >> v0) & 1)) {
        // new base w, a point of both cells: barycentric coordinates do not
        // depend on the base, so row(w) becomes the old base's coordinate
        // D - sum of the rows (a minor again) and the heights stay
        const int w = __builtin_ctzll(Cc & C);
        int64_t sum = 0;
#pragma unroll
        for (int r = 0; r < K; r++) sum += x[r];
        const int32_t xb = valid ? (int32_t)((int64_t)D - sum) : 0;
#pragma unroll
        for (int r = 0; r < K; r++)
          if (pivlane[r] == w) {
            x[r] = xb;
            pivlane[r] = v0;
          }
        v0 = w;
      }
      uint64_t outm = Cc & ~C, inm = C & ~Cc;
      bool ok = true;
      while (outm) {
        const int v = __builtin_ctzll(outm);
        outm &= outm - 1;
        int tp = 0;
        int32_t xr = 0;
#pragma unroll
        for (int r = 0; r < K; r++)
          if (pivlane[r] == v) {
            tp = r;
            xr = x[r];
          }
        const uint64_t cand = pballot(((inm >> lane) & 1) && xr != 0) & inm;
        if (!cand) {
          ok = false;
          break;
        }
        const int u = __builtin_ctzll(cand);
        inm &= ~(1ull << u);
        (void)pivot(tp, u);
      }
      elim = !ok;
    }
    if (elim) {
      v0 = __builtin_ctzll(C);
      // lane j's column: spatial differences and the split height difference
      H1 = H0 = 0;
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
        have = false;
        continue;
      }
      D = prev;
      Cc = C;
    }
    // The cell, then cells reached from it by pivots of the tableau instead
    // of new eliminations: depth first over new neighbours across facets
    // t < k (they keep the base point), returning to a cell by the inverse
    // pivot, at most `reach` cells per claimed cell.  A new neighbour that is
    // not reserved for a pivot goes to the list.
    uint32_t reach = item_reach;
    have = true; // (cleared when the cell is found not to be a lower facet)
    int depth = 0;
    bool fresh_cell = true; // false: back at a cell by the inverse pivot
    for (;;) {
      if (fresh_cell) {
        const bool neg = D < 0;
        const bool in_c = (Cc >> lane) & 1;
        // height above the cell's hyperplane, times |D|
        const int64_t s_raw = (int64_t)H1 * ((int64_t)1 << 31) + (int64_t)(uint32_t)H0;
        const int64_t S = neg ? -s_raw : s_raw;
        const bool other = valid && !in_c;
        const uint64_t below = pballot(other && S < 0), on = pballot(other && S == 0);
        if (below) { // not a lower facet: the start cell was wrong, or a bug
          if (lane == 0) atomicOr(&a.cnt->flags, PIVOT_ERR_STATE);
          have = false;
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
        // facets: opposite the point pivoted at step t (row t), then opposite
        // v0; lane t keeps the point entering across facet t (-1: none, the
        // facet is on the boundary of the hull) and the point leaving.  The
        // heights of the points beyond a facet are >= 0 (a point below has
        // ended the cell above), so each lane's ratio numerator is rounded
        // to float once for all facets.
        const float fS = ratio_num((uint64_t)(S > 0 ? S : 0));
        int my_u = -1, my_v = 0;
#pragma unroll
        for (int t = 0; t <= K; t++) {
          int32_t den; // lambda * |D| negated, for the points beyond the facet
          if (t < K) {
            const int32_t cs = neg ? -x[t] : x[t];
            den = other && cs < 0 ? -cs : 0;
          } else {
            const int64_t cs = neg ? -c0 : c0;
            den = other && cs < 0 ? (int32_t)(-cs) : 0;
          }
          const RatioMin rm = ratio_min_nonneg(fS, S, den);
          if ((rm.lanes & (rm.lanes - 1)) && lane == 0) atomicOr(&a.cnt->flags, PIVOT_TIE); // equal minima
          if (lane == t) {
            my_u = rm.lane;
            my_v = t < K ? pivlane[t] : v0;
          }
        }
        const uint64_t mine = my_u >= 0 ? (Cc & ~(1ull << my_v)) | (1ull << my_u) : 0ull;
        // lane t inserts the neighbour across facet t: all probes in one round
        const bool fresh = mine && set_insert(a, mine);
        // The level's room: `committed` holds the insertions made plus k + 1
        // for every cell committed and not yet processed, plus what the
        // waves hold as credit, and stays within a.room (the cells the set
        // and the list can still take).  This cell's unused insertions go
        // to the wave's credit; new neighbours across facets t < k are
        // reserved for pivots at k + 1 each, while this claimed cell's reach
        // and the credit allow.  A wave short of credit takes a chunk of the
        // level's room (one shared atomic per many cells).
        const uint64_t fb = pballot(fresh);
        const uint64_t fr = fb & ((1ull << K) - 1);
        credit += (uint32_t)(K + 1 - __builtin_popcountll(fb));
        const uint32_t want = min((uint32_t)__builtin_popcountll(fr), reach);
        if (want * (K + 1) > credit) {
          const uint32_t ask = max(want * (K + 1) - credit, (uint32_t)(PIVOT_CREDIT_CELLS * (K + 1)));
          const uint32_t before =
              (uint32_t)prl((int32_t)atomicAdd(&a.cnt->committed, lane == 0 ? ask : 0u), 0);
          const uint32_t fit = before >= a.room ? 0u : min(ask, a.room - before);
          if (fit < ask && lane == 0) atomicSub(&a.cnt->committed, ask - fit);
          credit += fit;
        }
        const uint32_t got = min(want, credit / (uint32_t)(K + 1));
        credit -= got * (uint32_t)(K + 1);
        constexpr uint32_t chunk = (uint32_t)(PIVOT_CREDIT_CELLS * (K + 1));
        if (credit > 4 * chunk) { // hand back what the wave does not need
          if (lane == 0) atomicSub(&a.cnt->committed, credit - chunk);
          credit = chunk;
        }
        uint64_t R = 0;
        {
          uint64_t f = fr;
          for (uint32_t i = 0; i < got; i++) {
            const uint64_t low = f & (~f + 1);
            R |= low;
            f ^= low;
          }
        }
        reach -= got;
        // the other new neighbours go to the list (through the wave's buffer)
        const uint64_t lm = fb & ~R;
        const uint32_t nl = (uint32_t)__builtin_popcountll(lm);
        if (nbuf + nl > 64u) flush();
        if ((lm >> lane) & 1) s_buf[wv][nbuf + __builtin_popcountll(lm & ((1ull << lane) - 1))] = mine;
        nbuf += nl;
        if ((R >> lane) & 1) s_u[wv][depth][lane] = (uint8_t)my_u;
        if (lane == 0) s_res[wv][depth] = (uint32_t)R;
      }
      // next: the deepest cell's next reserved neighbour, else back up one
      const uint32_t Rd = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)s_res[wv][depth]);
      int tp, up;
      if (Rd) {
        tp = __builtin_ctz(Rd);
        up = __builtin_amdgcn_readfirstlane((int32_t)s_u[wv][depth][tp]);
        if (lane == 0) s_res[wv][depth] = Rd & (Rd - 1);
      } else if (depth > 0) {
        tp = __builtin_amdgcn_readfirstlane((int32_t)s_row[wv][depth]);
        up = __builtin_amdgcn_readfirstlane((int32_t)s_left[wv][depth]);
      } else {
        break;
      }
      const int vout = pivot(tp, up);
      if (Rd) { // down into the reserved neighbour
        depth++;
        if (lane == 0) {
          s_row[wv][depth] = (uint8_t)tp;
          s_left[wv][depth] = (uint8_t)vout;
        }
        fresh_cell = true;
      } else { // back up
        depth--;
        fresh_cell = false;
      }
    }
  }
  if (nbuf) flush();
  // the credit goes back to the level's room, so that `committed` ends as
  // the number of cells the level inserted
  if (lane == 0 && credit) atomicSub(&a.cnt->committed, credit);
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
