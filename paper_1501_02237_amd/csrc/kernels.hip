// Device path of the degree computation on gfx950 (CDNA4, wave64).
//
// What is computed (paper Section 4): for every candidate (k+1)-subset
// {a_0..a_k} of the lifted points a^ = (a, w(a)), the hyperplane through the
// subset, its orientation, and whether every other lifted point lies strictly
// above it (eq. "lower-face", strict as in eq. "lower-d-face-again").  Lower
// facets add |det(a_1 - a_0, ..., a_k - a_0)| (eq. "simplex-vol"); a
// candidate with no point below and some point on the hyperplane is a tie
// (the lifting is not generic) and is flagged.
//
// How (designed for 64-lane wavefronts; no floating point, no MFMA):
//   * One wavefront owns one work unit: the candidates whose top elements
//     (colex order) are a fixed prefix, optionally restricted to a run of
//     sibling subtrees, completed downward by a depth-first walk.  Lane j holds
//     lifted point j (N <= 64); when N <= 32 (16, 8) the point set is
//     replicated in 2 (4, 8) lane groups.
//   * Walking down fixes one more point c: its residual row is broadcast with
//     v_readlane (wave-uniform scalars) and every lane eliminates it from its
//     own residual by one fraction-free (Bareiss) step,
//         r'_i = (piv * r_i - rc_i * r_p) / prev,
//     dividing exactly by the previous pivot through its 2-adic inverse.  After
//     t steps a lane's residuals are (t+1)x(t+1) minors of the chosen
//     difference rows bordered by its own point, so the work of a shared
//     prefix is done once for all candidates below it.  A chosen point whose
//     spatial residual vanishes makes every completion degenerate (D = 0): the
//     whole subtree is skipped.
//   * With k points fixed (a "ridge") a lane's residual is (sigma_j, h_j): one
//     spatial column and the height column.  Adding candidate c gives
//         D = sigma_c   (the k x k spatial determinant, up to a sign shared by
//                        every value of this ridge),
//         s_j * prev = sigma_c * h_j - h_c * sigma_j  (the (k+1)-minor with
//                        row j: point j's height over the hyperplane, times D),
//     so a candidate's lower-facet test is one 2x2 cross product per lane and a
//     wavefront ballot.  When the point set is replicated, each lane group
//     builds a different sibling ridge and tests that ridge's candidates.
//   * Heights are held as h = H1 * 2^31 + H0 (0 <= H0 < 2^31), so every
//     product is a signed 32 x 32 -> 64 multiply-add; the height residual and
//     the cross product are assembled from two 64-bit halves.  The host
//     certifies spatial minors < 2^31 and height minors < 2^60.
//   * Sums of |D| are kept per wavefront and added to the system's 128-bit
//     accumulator with 64-bit atomics and an explicit carry.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"

namespace bdeg {
namespace dev {

constexpr uint32_t LOW31 = 0x7FFFFFFFu;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- exact division
// divisor d = (-1)^neg * 2^e * odd; inv = (-1)^neg * odd^{-1} mod 2^64, so that
// an exact quotient is ((x >> e) * inv) mod 2^w.
struct Div {
  uint64_t inv;
  uint32_t e;
};

__device__ __forceinline__ Div make_div(int32_t d) {
  Div r;
  const uint32_t a = d < 0 ? (uint32_t)(-(int64_t)d) : (uint32_t)d;
  r.e = (uint32_t)__builtin_ctz(a);
  const uint32_t odd = a >> r.e;
  uint32_t x = odd; // odd * odd == 1 mod 8: 3 correct bits, doubled by each Newton step
  x *= 2u - odd * x;  // 6
  x *= 2u - odd * x;  // 12
  x *= 2u - odd * x;  // 24
  x *= 2u - odd * x;  // 48 -> 32 bits correct
  uint64_t y = x;
  y *= 2ull - (uint64_t)odd * y; // 64 bits correct
  r.inv = d < 0 ? (uint64_t)0 - y : y;
  return r;
}

// x is an exact multiple of the divisor and the quotient fits int32.
__device__ __forceinline__ int32_t exdiv32(int64_t x, const Div &d) {
  return (int32_t)((uint32_t)((uint64_t)x >> d.e) * (uint32_t)d.inv);
}
// (A * 2^31 + B) / d for an exact multiple whose quotient fits int64; e <= 30.
__device__ __forceinline__ int64_t exdiv_split(int64_t A, int64_t B, const Div &d) {
  const uint64_t y = ((uint64_t)A << (31 - d.e)) + (uint64_t)(B >> d.e);
  return (int64_t)(y * d.inv);
}

// ---------------------------------------------------------------- cross-lane helpers
__device__ __forceinline__ int32_t rl32(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int32_t bp32(int32_t v, int src_lane) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// ---------------------------------------------------------------- per-wave state
// A state of depth t keeps only its pivot as a scalar; the pivot's 2-adic
// inverse is recomputed where it is used, so that no per-level scalar data
// stays live across the deeper levels (the scalar register file is small).
template <int W>
struct St {
  int32_t s[W > 0 ? W : 1]; // spatial residuals (W columns)
  int32_t H1, H0;           // height residual h = H1 * 2^31 + H0
  int32_t prev;             // the pivot that produced this state
};

template <bool S> // S: count work (profiling variant)
struct Ctx {
  int npl;              // log2 of lanes per point group
  int G;                // point groups in the wave
  int g, j;             // this lane's group and point
  uint64_t mask;        // work unit prefix
  int L;                // prefix length
  int c_lo, c_hi;       // sibling run at the first free level
  uint64_t valid_lanes; // lanes holding a real point, all groups
  uint64_t rep_unit;    // bit 0 of every group
  uint64_t rep_diag;    // bit q*(npad-1) for every group q
  uint64_t chosen_rep;  // chosen points, replicated in every group
  uint64_t acc;         // sum of |D| of lower facets in this unit
  uint32_t cells, tie;
  // watchdog: loop steps left for this unit (a budget derived from the unit's
  // candidate count); running out abandons the unit and reports a device
  // error, so no wavefront can loop without end
  uint32_t left;
  // work counters of the profiling variant
  uint32_t leaves, ridges, inner, sp_upd, pruned;
};

template <bool S>
__device__ __forceinline__ bool step_ok(Ctx<S> &cx) {
  if (cx.left == 0) return false;
  cx.left--;
  return true;
}

__device__ __forceinline__ uint64_t binom_dev(int n, int r) {
  if (r < 0 || r > n) return 0;
  uint64_t c = 1;
  for (int i = 1; i <= r; i++) c = c * (uint64_t)(n - r + i) / (uint64_t)i;
  return c;
}

// candidates of a work unit (prefix with L elements, lowest e, run [c_lo, c_hi])
__device__ __forceinline__ uint64_t unit_candidates(int k, uint64_t mask, int c_lo, int c_hi) {
  const int L = __builtin_popcountll(mask);
  if (L >= k + 1) return 1;
  const int e = __builtin_ctzll(mask);
  const int i = k - L; // colex position of the next element
  const int hi = min(e - 1, c_hi), lo = max(i, c_lo);
  if (hi < lo) return 0;
  return binom_dev(hi + 1, i + 1) - binom_dev(lo, i + 1);
}

// Bit of point x - q in group q, for groups q < ng: the replicated diagonal
// (bit q*(npad-1) of rep_diag) restricted to those groups BEFORE the shift, so
// that a group without a candidate contributes no bit (its bit would land in
// the group below it).
template <bool S>
__device__ __forceinline__ uint64_t diag_bits(const Ctx<S> &cx, int x, int ng) {
  const int top = (ng - 1) * ((1 << cx.npl) - 1); // position of the last kept bit
  return (cx.rep_diag & ((2ull << top) - 1)) << x;
}

// Fetch a value of point `c - g` of this lane's group, where the group's
// candidate is c - g (uniform readlane when the wave has one group).
template <bool S>
__device__ __forceinline__ int32_t fetch_diag(const Ctx<S> &cx, int32_t v, int c, int src) {
  return cx.G == 1 ? rl32(v, c) : bp32(v, src);
}

// Decide the candidates of one leaf step, one per group q < ngroups (the
// candidate of group q is point cand_lane0 - q of that group).
template <bool S>
__device__ __forceinline__ void decide(Ctx<S> &cx, uint64_t m_neg, uint64_t m_nz, uint64_t m_sc, uint64_t active,
                                       int32_t sig, int cand_lane0, int ngroups) {
  const uint64_t neg = m_neg & active;
  const uint64_t zero = ~m_nz & active;
  const int npad = 1 << cx.npl;
  const uint64_t gm0 = npad == 64 ? ~0ull : ((1ull << npad) - 1);
  for (int q = 0; q < ngroups; q++) {
    const uint64_t gm = gm0 << (q << cx.npl);
    if (!(m_sc & gm)) continue; // no candidate or D = 0 in this group
    if constexpr (S) cx.leaves++;
    if (neg & gm) continue;
    if (zero & gm) {
      cx.tie = 1;
      continue;
    }
    const int32_t sv = rl32(sig, (q << cx.npl) + cand_lane0 - q);
    cx.acc += (uint64_t)(sv < 0 ? -(int64_t)sv : (int64_t)sv);
    cx.cells++;
  }
}

// Sign pieces of t = sc * h_j - hc * sig_j with h = H1 * 2^31 + H0:
// t = 2^31 * C + Blo with C = A + (B >> 31), Blo = B mod 2^31.
struct Cross {
  bool lt, nz;
};
__device__ __forceinline__ Cross cross_sign(int32_t sc, int32_t h1c, int32_t h0c, int32_t sig, int32_t H1,
                                            int32_t H0) {
  const int64_t A = (int64_t)sc * H1 - (int64_t)h1c * sig;
  const int64_t B = (int64_t)sc * H0 - (int64_t)h0c * sig;
  const int64_t C = A + (B >> 31);
  const uint32_t Blo = (uint32_t)B & LOW31;
  Cross r;
  r.lt = C < 0;
  r.nz = (C != 0) | (Blo != 0);
  return r;
}

// Leaves of one ridge whose state is identical in every group: the groups
// test consecutive candidates c, c-1, ... of the ridge in one step.
template <bool S>
__device__ __forceinline__ void leaves_uniform(Ctx<S> &cx, const St<1> &st, int hi_c, int lo_c) {
  const int G = cx.G;
  const int32_t sig = st.s[0], H1 = st.H1, H0 = st.H0;
  const bool prevneg = st.prev < 0;
  for (int c0 = hi_c; c0 >= lo_c && step_ok(cx); c0 -= G) {
    const int cg = c0 - cx.g;
    const bool ok = cg >= lo_c;
    const int src = (cx.g << cx.npl) + (ok ? cg : 0);
    const int32_t sc = fetch_diag(cx, sig, c0, src);
    const int32_t h1c = fetch_diag(cx, H1, c0, src);
    const int32_t h0c = fetch_diag(cx, H0, c0, src);
    const Cross t = cross_sign(sc, h1c, h0c, sig, H1, H0);
    const bool flip = (sc < 0) != prevneg;
    const uint64_t m_neg = ballot(t.nz && (t.lt != flip));
    const uint64_t m_nz = ballot(t.nz);
    const uint64_t m_sc = ballot(ok && sc != 0);
    const int ng = min(G, c0 - lo_c + 1);
    const uint64_t active = cx.valid_lanes & ~cx.chosen_rep & ~diag_bits(cx, c0, ng) & m_sc;
    decide(cx, m_neg, m_nz, m_sc, active, sig, c0, ng);
  }
}

// Range of the next element at depth T (T+1 points chosen, lowest `low`).
template <bool S>
__device__ __forceinline__ bool next_range(const Ctx<S> &cx, int T, int K, int low, int *hi_c, int *lo_c) {
  if (T + 1 < cx.L) { // fixed by the work unit's prefix
    const uint64_t below = cx.mask & ((1ull << low) - 1);
    *hi_c = *lo_c = 63 - __builtin_clzll(below);
    return true;
  }
  *hi_c = low - 1;
  *lo_c = K - T - 1;
  if (T + 1 == cx.L) { // sibling run of the work unit
    *hi_c = min(*hi_c, cx.c_hi);
    *lo_c = max(*lo_c, cx.c_lo);
  }
  return false;
}

// st holds depth T (T+1 points chosen, lowest `low`).
template <int K, int T, bool S>
struct Level {
  static __device__ __forceinline__ void run(Ctx<S> &cx, const St<K - T> &st, int low) {
    constexpr int W = K - T;
    int hi_c, lo_c;
    const bool forced = next_range(cx, T, K, low, &hi_c, &lo_c);
    if constexpr (T + 2 < K) {
      // create a node of depth T+1 < k-1 (uniform state, readlane broadcast)
      for (int c = hi_c; c >= lo_c && step_ok(cx); --c) {
        int32_t rc[W];
#pragma unroll
        for (int i = 0; i < W; i++) rc[i] = rl32(st.s[i], c);
        int p = -1;
#pragma unroll
        for (int i = 0; i < W; i++)
          if (p < 0 && rc[i] != 0) p = i;
        if (p < 0) { // the new point is affinely dependent on the prefix: D = 0 below
          if constexpr (S) cx.pruned++;
          continue;
        }
        int32_t piv = rc[0], rjp = st.s[0];
#pragma unroll
        for (int i = 1; i < W; i++)
          if (p == i) {
            piv = rc[i];
            rjp = st.s[i];
          }
        const int32_t h1c = rl32(st.H1, c), h0c = rl32(st.H0, c);
        const Div dv = make_div(st.prev); // dead before the recursion below
        St<W - 1> ch;
#pragma unroll
        for (int i = 0; i < W - 1; i++) {
          const bool sh = i >= p;
          const int32_t src = sh ? st.s[i + 1] : st.s[i];
          const int32_t rcs = sh ? rc[i + 1] : rc[i];
          ch.s[i] = exdiv32((int64_t)piv * src - (int64_t)rcs * rjp, dv);
        }
        const int64_t A = (int64_t)piv * st.H1 - (int64_t)h1c * rjp;
        const int64_t B = (int64_t)piv * st.H0 - (int64_t)h0c * rjp;
        const int64_t h = exdiv_split(A, B, dv);
        ch.H1 = (int32_t)(h >> 31);
        ch.H0 = (int32_t)((uint32_t)h & LOW31);
        ch.prev = piv;
        cx.chosen_rep |= cx.rep_unit << c;
        if constexpr (S) {
          cx.inner++;
          cx.sp_upd += W - 1;
        }
        Level<K, T + 1, S>::run(cx, ch, c);
        cx.chosen_rep &= ~(cx.rep_unit << c);
      }
    } else {
      // T = k-2: create ridges (depth k-1) from a 2-column state, then test
      // their candidates.
      static_assert(W == 2, "ridge level");
      const Div dv = make_div(st.prev);
      if (forced || cx.G == 1) {
        // one ridge at a time; groups share its candidates
        for (int c = hi_c; c >= lo_c && step_ok(cx); --c) {
          const int32_t r0 = rl32(st.s[0], c), r1 = rl32(st.s[1], c);
          if (r0 == 0 && r1 == 0) {
            if constexpr (S) cx.pruned++;
            continue;
          }
          const bool p0 = r0 != 0;
          const int32_t piv = p0 ? r0 : r1, rco = p0 ? r1 : r0;
          const int32_t rjp = p0 ? st.s[0] : st.s[1], so = p0 ? st.s[1] : st.s[0];
          const int32_t h1c = rl32(st.H1, c), h0c = rl32(st.H0, c);
          St<1> r;
          r.s[0] = exdiv32((int64_t)piv * so - (int64_t)rco * rjp, dv);
          const int64_t A = (int64_t)piv * st.H1 - (int64_t)h1c * rjp;
          const int64_t B = (int64_t)piv * st.H0 - (int64_t)h0c * rjp;
          const int64_t h = exdiv_split(A, B, dv);
          r.H1 = (int32_t)(h >> 31);
          r.H0 = (int32_t)((uint32_t)h & LOW31);
          r.prev = piv;
          if constexpr (S) cx.ridges++;
          cx.chosen_rep |= cx.rep_unit << c;
          int lhi = c - 1, llo = 0;
          if (T + 2 < cx.L) { // the candidate itself is fixed (rank-range units)
            const uint64_t below = cx.mask & ((1ull << c) - 1);
            lhi = llo = 63 - __builtin_clzll(below);
          } else if (T + 2 == cx.L) {
            lhi = min(lhi, cx.c_hi);
            llo = max(llo, cx.c_lo);
          }
          leaves_uniform(cx, r, lhi, llo);
          cx.chosen_rep &= ~(cx.rep_unit << c);
        }
      } else {
        // each lane group builds its own sibling ridge c - g and tests it
        const int G = cx.G;
        for (int c = hi_c; c >= lo_c && step_ok(cx); c -= G) {
          const int cg = c - cx.g;
          const bool gok = cg >= lo_c;
          const int src = (cx.g << cx.npl) + (gok ? cg : 0);
          const int32_t r0 = bp32(st.s[0], src), r1 = bp32(st.s[1], src);
          const int32_t h1c = bp32(st.H1, src), h0c = bp32(st.H0, src);
          const bool p0 = r0 != 0;
          const bool alive = gok && (p0 || r1 != 0);
          const int32_t piv = p0 ? r0 : (r1 != 0 ? r1 : 1);
          const int32_t rco = p0 ? r1 : r0;
          const int32_t rjp = p0 ? st.s[0] : st.s[1], so = p0 ? st.s[1] : st.s[0];
          const int32_t sig = exdiv32((int64_t)piv * so - (int64_t)rco * rjp, dv);
          const int64_t A = (int64_t)piv * st.H1 - (int64_t)h1c * rjp;
          const int64_t B = (int64_t)piv * st.H0 - (int64_t)h0c * rjp;
          const int64_t h = exdiv_split(A, B, dv);
          const int32_t H1 = (int32_t)(h >> 31), H0 = (int32_t)((uint32_t)h & LOW31);
          const bool pivneg = piv < 0;
          const uint64_t m_alive = ballot(alive);
          const int ngr = min(G, c - lo_c + 1);
          if constexpr (S) {
            const uint32_t n_alive = (uint32_t)__builtin_popcountll(m_alive & cx.rep_unit);
            cx.ridges += n_alive;
            cx.pruned += (uint32_t)ngr - n_alive;
          }
          if (!m_alive) continue;
          const uint64_t chosen_g = cx.chosen_rep | diag_bits(cx, c, ngr);
          // candidates: group q tests cc - q for cc = c-1 .. 0
          for (int cc = c - 1; cc >= 0 && step_ok(cx); --cc) {
            const int cq = cc - cx.g;
            const bool lok = cq >= 0;
            const int src2 = (cx.g << cx.npl) + (lok ? cq : 0);
            const int32_t sc = bp32(sig, src2), hc1 = bp32(H1, src2), hc0 = bp32(H0, src2);
            const Cross t = cross_sign(sc, hc1, hc0, sig, H1, H0);
            const bool flip = (sc < 0) != pivneg;
            const uint64_t m_neg = ballot(t.nz && (t.lt != flip));
            const uint64_t m_nz = ballot(t.nz);
            const uint64_t m_sc = ballot(lok && alive && sc != 0);
            const int ng = min(ngr, cc + 1);
            const uint64_t active = cx.valid_lanes & ~chosen_g & ~diag_bits(cx, cc, ng) & m_sc;
            decide(cx, m_neg, m_nz, m_sc, active, sig, cc, ng);
          }
        }
      }
    }
  }
};

template <int K, bool S>
__device__ __forceinline__ void process_tile(Ctx<S> &cx, const SysDesc &sd, const int32_t *__restrict__ pts,
                                             const int64_t *__restrict__ hts) {
  const bool valid = cx.j < sd.N;
  int32_t P[K];
  int64_t w = 0;
#pragma unroll
  for (int i = 0; i < K; i++) P[i] = 0;
  if (valid) {
#pragma unroll
    for (int i = 0; i < K; i++) P[i] = pts[sd.pt_off + cx.j * K + i];
    w = hts[sd.ht_off + cx.j];
  }
  const int base = 63 - __builtin_clzll(cx.mask);
  const int64_t wb = (int64_t)(((uint64_t)(uint32_t)rl32((int32_t)(uint32_t)((uint64_t)w >> 32), base) << 32) |
                               (uint32_t)rl32((int32_t)(uint32_t)w, base));
  const int64_t h0 = w - wb;
  St<K> st;
#pragma unroll
  for (int i = 0; i < K; i++) st.s[i] = P[i] - rl32(P[i], base);
  st.H1 = (int32_t)(h0 >> 31);
  st.H0 = (int32_t)((uint32_t)h0 & LOW31);
  st.prev = 1;
  cx.chosen_rep = cx.rep_unit << base;
  if constexpr (K == 1) {
    // the base point alone is the ridge
    int hi = base - 1, lo = 0;
    if (cx.L >= 2) {
      const uint64_t below = cx.mask & ((1ull << base) - 1);
      hi = lo = 63 - __builtin_clzll(below);
    } else {
      hi = min(hi, cx.c_hi);
      lo = max(lo, cx.c_lo);
    }
    St<1> r;
    r.s[0] = st.s[0];
    r.H1 = st.H1;
    r.H0 = st.H0;
    r.prev = 1;
    if constexpr (S) cx.ridges++;
    leaves_uniform(cx, r, hi, lo);
  } else {
    Level<K, 0, S>::run(cx, st, base);
  }
}

template <int KLO, int KHI, bool S>
__global__ void __launch_bounds__(256) enum_kernel(const SysDesc *__restrict__ sys,
                                                   const int32_t *__restrict__ pts,
                                                   const int64_t *__restrict__ hts,
                                                   const Tile *__restrict__ tiles, uint32_t n_tiles,
                                                   SysAcc *__restrict__ acc, DevCounters *__restrict__ cnt) {
  const int lane = lane_id();
  Ctx<S> cx;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&cnt->next_tile, 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= n_tiles) break;
    const Tile tl = tiles[t];
    const SysDesc sd = sys[tl.sys];
    cx.npl = sd.npad_log2;
    cx.G = 64 >> sd.npad_log2;
    cx.g = lane >> sd.npad_log2;
    cx.j = lane & ((1 << sd.npad_log2) - 1);
    cx.mask = tl.mask;
    cx.L = __builtin_popcountll(tl.mask);
    cx.c_lo = tl.c_lo;
    cx.c_hi = tl.c_hi;
    uint64_t unit = 0, vl = 0, diag = 0;
    const uint64_t pm = sd.N >= 64 ? ~0ull : ((1ull << sd.N) - 1);
    for (int q = 0; q < cx.G; q++) {
      unit |= 1ull << (q << sd.npad_log2);
      diag |= 1ull << ((q << sd.npad_log2) - q);
      vl |= pm << (q << sd.npad_log2);
    }
    cx.rep_unit = unit;
    cx.rep_diag = diag;
    cx.valid_lanes = vl;
    cx.acc = 0;
    cx.cells = 0;
    cx.tie = 0;
    cx.leaves = cx.ridges = cx.inner = cx.sp_upd = cx.pruned = 0;
    {
      // every loop step of a unit is charged to a candidate below it, and a
      // candidate is charged at most once per depth: k + 1 steps suffice
      const uint64_t cand = unit_candidates(sd.k, tl.mask, tl.c_lo, tl.c_hi);
      const uint64_t b = cand * (uint64_t)(sd.k + 3) + 256;
      cx.left = b > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)b;
    }
    switch (sd.k) {
#define BDEG_CASE(KK)                                      \
  case KK:                                                 \
    if constexpr (KK >= KLO && KK <= KHI)                  \
      process_tile<KK, S>(cx, sd, pts, hts);               \
    break;
      BDEG_CASE(1) BDEG_CASE(2) BDEG_CASE(3) BDEG_CASE(4) BDEG_CASE(5) BDEG_CASE(6)
      BDEG_CASE(7) BDEG_CASE(8) BDEG_CASE(9) BDEG_CASE(10) BDEG_CASE(11) BDEG_CASE(12)
#undef BDEG_CASE
      default:
        break;
    }
    const bool abandoned = cx.left == 0;
    if (lane == 0 && abandoned) atomicOr(&cnt->error, 1u);
    if (lane == 0 && !abandoned) {
      if (cx.acc | cx.cells | cx.tie) {
        SysAcc *a = &acc[tl.sys];
        const unsigned long long old = atomicAdd((unsigned long long *)&a->lo, (unsigned long long)cx.acc);
        if (old + cx.acc < old) atomicAdd((unsigned long long *)&a->hi, 1ull);
        atomicAdd((unsigned long long *)&a->cells, (unsigned long long)cx.cells);
        if (cx.tie) atomicOr(&a->tie, 1u);
      }
      if constexpr (S) {
        atomicAdd((unsigned long long *)&cnt->ridges, (unsigned long long)cx.ridges);
        atomicAdd((unsigned long long *)&cnt->inner, (unsigned long long)cx.inner);
        atomicAdd((unsigned long long *)&cnt->sp_upd, (unsigned long long)cx.sp_upd);
        atomicAdd((unsigned long long *)&cnt->leaves, (unsigned long long)cx.leaves);
        atomicAdd((unsigned long long *)&cnt->pruned, (unsigned long long)cx.pruned);
        atomicAdd((unsigned long long *)&cnt->tiles, 1ull);
      }
    }
  }
}

// heights of the listed systems (all systems when active == nullptr)
__global__ void lift_kernel(const SysDesc *__restrict__ sys, const int32_t *__restrict__ active, int n_active,
                            int64_t *__restrict__ hts) {
  const int s = blockIdx.x;
  if (s >= n_active) return;
  const int sid = active ? active[s] : s;
  const SysDesc d = sys[sid];
  const int j = threadIdx.x;
  if (j < d.N) {
    const uint64_t z = mix64(d.lift_key + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull);
    hts[d.ht_off + j] = (int64_t)(z >> (64 - d.lift_bits));
  }
}

__global__ void clear_kernel(SysAcc *__restrict__ acc, int n_sys, DevCounters *__restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_sys) {
    acc[i].lo = 0;
    acc[i].hi = 0;
    acc[i].cells = 0;
    acc[i].tie = 0;
    acc[i].pad = 0;
  }
  if (i == 0 && cnt) {
    cnt->ridges = cnt->inner = cnt->sp_upd = cnt->pruned = cnt->leaves = cnt->tiles = 0;
    cnt->next_tile = 0;
    cnt->error = 0;
  }
}

// clear the partial sums of the listed systems
__global__ void clear_list_kernel(SysAcc *__restrict__ acc, const int32_t *__restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    SysAcc *a = &acc[list[i]];
    a->lo = 0;
    a->hi = 0;
    a->cells = 0;
    a->tie = 0;
    a->pad = 0;
  }
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

int launch_clear(void *stream, SysAcc *d_acc, int n_sys, DevCounters *d_cnt) {
  int n = n_sys > 1 ? n_sys : 1;
  hipLaunchKernelGGL(dev::clear_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_acc, n_sys,
                     d_cnt);
  return hip_ok(hipGetLastError());
}

int launch_clear_list(void *stream, SysAcc *d_acc, const int32_t *d_list, int n) {
  if (n <= 0) return BDEG_OK;
  hipLaunchKernelGGL(dev::clear_list_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_acc, d_list,
                     n);
  return hip_ok(hipGetLastError());
}

typedef void (*EnumFn)(const SysDesc *, const int32_t *, const int64_t *, const Tile *, uint32_t, SysAcc *,
                       DevCounters *);

// Single-k kernels (exact register budget) and mixed-k kernels for batches;
// `stats` selects the variant that also counts its work.
template <bool S>
static EnumFn enum_fn_s(int klo, int khi) {
  if (klo == khi) {
    switch (khi) {
      case 1: return dev::enum_kernel<1, 1, S>;
      case 2: return dev::enum_kernel<2, 2, S>;
      case 3: return dev::enum_kernel<3, 3, S>;
      case 4: return dev::enum_kernel<4, 4, S>;
      case 5: return dev::enum_kernel<5, 5, S>;
      case 6: return dev::enum_kernel<6, 6, S>;
      case 7: return dev::enum_kernel<7, 7, S>;
      case 8: return dev::enum_kernel<8, 8, S>;
      case 9: return dev::enum_kernel<9, 9, S>;
      case 10: return dev::enum_kernel<10, 10, S>;
      case 11: return dev::enum_kernel<11, 11, S>;
      case 12: return dev::enum_kernel<12, 12, S>;
      default: return nullptr;
    }
  }
  if (khi <= 7) return dev::enum_kernel<1, 7, S>;
  if (khi <= 12) return dev::enum_kernel<1, 12, S>;
  return nullptr;
}

static EnumFn enum_fn(int klo, int khi, bool stats) {
  return stats ? enum_fn_s<true>(klo, khi) : enum_fn_s<false>(klo, khi);
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

int max_enum_blocks(int klo, int khi, int waves_per_block) {
  EnumFn f = enum_fn(klo, khi, false);
  if (!f) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)f, waves_per_block * 64, 0) != hipSuccess)
    return 0;
  return per_cu * device_cu_count();
}

int launch_enumerate(void *stream, const SysDesc *d_sys, const int32_t *d_pts, const int64_t *d_heights,
                     const Tile *d_tiles, uint32_t n_tiles, SysAcc *d_acc, DevCounters *d_cnt, int klo, int khi,
                     LaunchShape shape) {
  EnumFn f = enum_fn(klo, khi, shape.stats);
  if (!f) return BDEG_E_TOO_LARGE;
  if (n_tiles == 0) return BDEG_OK;
  int blocks = shape.blocks;
  const int wpb = shape.waves_per_block > 0 ? shape.waves_per_block : 4;
  if (blocks <= 0) blocks = max_enum_blocks(klo, khi, wpb);
  if (blocks <= 0) return BDEG_E_DEVICE;
  const uint64_t need = ((uint64_t)n_tiles + wpb - 1) / wpb;
  if ((uint64_t)blocks > need) blocks = (int)need;
  hipLaunchKernelGGL(f, dim3(blocks), dim3(wpb * 64), 0, (hipStream_t)stream, d_sys, d_pts, d_heights, d_tiles,
                     n_tiles, d_acc, d_cnt);
  return hip_ok(hipGetLastError());
}

} // namespace bdeg
