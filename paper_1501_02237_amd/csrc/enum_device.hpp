// Device code of the enumeration kernel (included by the per-k translation
// units, which instantiate it; see kernels.hip for the launch helpers).
#pragma once
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
#include "exact_div.hpp"

namespace bdeg {
namespace dev {

constexpr uint32_t LOW31 = 0x7FFFFFFFu;


// ---------------------------------------------------------------- cross-lane helpers
__device__ __forceinline__ int32_t rl32(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int32_t bp32(int32_t v, int src_lane) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
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

// Per-wave results of the current work unit (in LDS, written by lane 0).
struct Tally {
  unsigned long long acc; // sum of |D| over lower facets
  uint32_t cells;         // lower facets
  uint32_t tie;           // a non-generic lower face was seen
};

// MODE: MODE_PLAIN, MODE_STATS (also count the work) or MODE_EMIT (also list
// every lower facet found).  GG = 1: one point group fills the wave (N > 32),
// a compile-time fact that removes the sibling-ridge path and turns gathers
// into broadcasts.  GG = 0: the group count 64 / npad is read from the system
// descriptor at run time.
template <int MODE, int GG>
struct Ctx {
  static_assert(GG == 0 || GG == 1, "group specialisations");
  static constexpr bool single = GG == 1;
  static constexpr bool stats = MODE == MODE_STATS;
  static constexpr bool emit = MODE == MODE_EMIT;
  int npl_;             // log2 of lanes per point group (GG == 0)
  int G_;               // point groups in the wave (GG == 0)
  __device__ __forceinline__ int npl() const {
    if constexpr (single) return 6;
    else return npl_;
  }
  __device__ __forceinline__ int G() const {
    if constexpr (single) return 1;
    else return G_;
  }
  __device__ __forceinline__ int npad() const { return 1 << npl(); }
  int g, j;             // this lane's group and point
  uint64_t mask;        // work unit prefix
  int L;                // prefix length
  int c_lo, c_hi;       // sibling run at the first free level
  int jg;               // j + g: lane j of group g holds the candidate c - g when jg == c
  uint64_t valid_lanes; // lanes holding a real point, all groups
  uint64_t rep_unit;    // bit 0 of every group
  uint64_t top_bits;    // bit npad-1 of every group (the groups' bit fields)
  uint64_t chosen_rep;  // chosen points, replicated in every group
  // the unit's sum of |D| over lower facets, cell count and tie flag live in
  // a per-wave LDS slot: they change only when a cell is found, and kept in
  // registers they would be copied at every level of the loop nest
  struct Tally *tally;
  // watchdog: loop steps left for this unit (a budget derived from the unit's
  // candidate count); running out (left <= 0) abandons the unit and reports a
  // device error, so no wavefront can loop without end.  Signed, so that a
  // charge is a scalar subtract and a sign test (an unsigned saturating
  // subtract would go through a vector register)
  int32_t left;
  // work counters of the profiling variant
  uint32_t leaves, ridges, inner, sp_upd, pruned, rsteps, lsteps, lempty;
  // cell list of the emitting variant
  CellSink sink;
};

// point mask of group 0's lanes (the chosen set seen from one group)
template <class CX>
__device__ __forceinline__ uint64_t group0_mask(const CX &cx) {
  if constexpr (CX::single) return ~0ull;
  else return (1ull << cx.npad()) - 1;
}

// Append one lower facet (vertex mask) to the cell list; one lane per wave.
// Facets beyond the capacity are counted but not stored.
template <class CX>
__device__ __forceinline__ void emit_cell(CX &cx, uint64_t vertices) {
  if (lane_id() == 0) {
    const unsigned long long i = atomicAdd((unsigned long long *)cx.sink.count, 1ull);
    if (i < cx.sink.cap) cx.sink.masks[i] = vertices;
  }
}

template <class CX>
__device__ __forceinline__ bool step_ok(CX &cx) {
  if (cx.left <= 0) return false;
  cx.left--;
  return true;
}

// Charge the n steps of a leaf loop at once (the loop itself then runs
// without per-step checks); false when the budget cannot cover them, which
// abandons the unit like an exhausted step_ok.
template <class CX>
__device__ __forceinline__ bool charge(CX &cx, int n) {
  if (n <= 0) return true;
  cx.left -= n;
  return cx.left > 0;
}

// Binomial coefficients C(n, r), n <= 64, r <= BDEG_MAX_K + 1, as a Pascal
// triangle built at compile time (a unit's budget needs two per unit; a
// multiplicative loop would be a chain of 64-bit divisions)
constexpr int BINOM_R = BDEG_MAX_K + 2;
struct BinomTable {
  uint64_t v[65][BINOM_R];
};
constexpr BinomTable make_binom_table() {
  BinomTable t{};
  for (int n = 0; n <= 64; n++) {
    t.v[n][0] = 1;
    for (int r = 1; r < BINOM_R; r++) t.v[n][r] = n == 0 ? 0 : t.v[n - 1][r - 1] + t.v[n - 1][r];
  }
  return t;
}
static __constant__ BinomTable kBinom = make_binom_table();
__device__ __forceinline__ uint64_t binom_dev(int n, int r) {
  if (r < 0 || r > n) return 0;
  return kBinom.v[n][r]; // callers keep n <= 64 and r <= BDEG_MAX_K + 1
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

// Lanes j of every group g with j + g == c: the group's point c - g (its
// candidate, or its ridge point); no lane where c - g < 0.
template <class CX>
__device__ __forceinline__ uint64_t diag_lanes(const CX &cx, int c) {
  if constexpr (CX::single) return 1ull << c;
  else return ballot(cx.jg == c);
}

// The lane groups are bit fields of a wave mask (top_bits marks the top bit of
// each).  any_group(t) sets the top bit of every group in which t has a set
// bit: adding the group's low-bit mask to its low bits of t carries into the
// top bit exactly when one of them is set, and never past the group.
template <class CX>
__device__ __forceinline__ uint64_t any_group(const CX &cx, uint64_t t) {
  if constexpr (CX::single) return t ? cx.top_bits : 0ull;
  else return (((t & ~cx.top_bits) + ~cx.top_bits) | t) & cx.top_bits;
}

// Fetch a value of point `c - g` of this lane's group, where the group's
// candidate is c - g (uniform readlane when the wave has one group).
template <class CX>
__device__ __forceinline__ int32_t fetch_diag(const CX &cx, int32_t v, int c, int src) {
  if constexpr (CX::single)
    return rl32(v, c);
  else
    return bp32(v, src);
}

// Leaf test in sign-normalised form.  Each lane keeps a candidate view of its
// point j at the current ridge: a_j = sign(prev) |sigma_j| and the negated
// b_j = sign(prev) sign(sigma_j) h_j (both height halves, stored as -b_j so
// that each half of the cross product is a chain of multiply-adds).  For
// candidate c (D = sigma_c) and point j,
//     t' = a_c h_j - b_c sigma_j = sign(D prev) (sigma_c h_j - h_c sigma_j),
// whose sign is that of D s_j: point j lies below the candidate's hyperplane
// exactly when t' < 0.  With h = H1 2^31 + H0, t' = 2^31 C + lo, 0 <= lo < 2^31,
// so t' < 0 exactly when C < 0, and t' = 0 exactly when C = lo = 0.  With
// |a|, |sigma| < 2^31, 0 <= H0 < 2^31 and |H1| < 2^29 (height minors < 2^60)
// every partial sum below stays under 2^63.
struct View {
  int32_t a, nb1, nb0;
};
__device__ __forceinline__ View cand_view(int32_t sig, int32_t H1, int32_t H0, bool prevneg) {
  const int32_t mag = sig < 0 ? -sig : sig;
  const bool f = (sig < 0) != prevneg;
  View v;
  v.a = prevneg ? -mag : mag;
  v.nb1 = f ? H1 : -H1;
  v.nb0 = f ? H0 : -H0;
  return v;
}
struct Cross {
  int64_t C;
  uint32_t lo;
};
// t' = a h - b sigma from a, -b (both halves) and this lane's (sigma, H1, H0)
__device__ __forceinline__ Cross cross_view(int32_t a, int32_t nb1, int32_t nb0, int32_t sig, int32_t H1,
                                            int32_t H0) {
  const int64_t B = (int64_t)a * H0 + (int64_t)nb0 * sig;
  Cross r;
  r.C = (int64_t)a * H1 + ((int64_t)nb1 * sig + (B >> 31));
  r.lo = (uint32_t)B & LOW31;
  return r;
}

// Decide one leaf step: group q tests its candidate, point cand - q.
//   m_neg lanes strictly below their group's candidate hyperplane.  No lane
//         needs masking out: padding lanes and the chosen points and the
//         group's ridge point have vanishing residuals, and the candidate's own
//         cross product cancels, so their t' is exactly 0.
//   t     this lane's t' (for the zero test, needed only when a group survives)
//   has   top bits of the groups whose candidate exists and has D != 0
//   excl  lanes outside the zero test (padding, chosen points, ridge points);
//         the candidates' own lanes are added only when a group survives
// A group with a point strictly below the candidate's hyperplane rejects
// (the common case, decided for all groups with a handful of scalar mask
// operations); otherwise a point on the hyperplane is a tie and none is a
// lower facet.  For the cell list: `fixed` holds the points every group
// shares and, when ridge >= 0, group q's ridge adds point ridge - q.
template <class CX>
__device__ __forceinline__ void decide(CX &cx, uint64_t m_neg, const Cross &t, uint64_t has, uint64_t excl,
                                       int32_t sig, int cand, uint64_t fixed, int ridge) {
  if constexpr (CX::stats) {
    cx.leaves += (uint32_t)__builtin_popcountll(has);
    cx.lsteps++;
    cx.lempty += has == 0;
  }
  const uint64_t ok = has & ~any_group(cx, m_neg);
  if (ok == 0) return;
  excl |= diag_lanes(cx, cand);
  const uint64_t m_nz = ballot((t.C != 0) | (t.lo != 0));
  const uint64_t zero = ok & any_group(cx, ~(m_nz | excl));
  const int npl = cx.npl();
  uint64_t add = 0;
  uint32_t found = 0;
  for (uint64_t a = ok & ~zero; a; a &= a - 1) {
    const int q = __builtin_ctzll(a) >> npl;
    const int32_t sv = rl32(sig, (q << npl) + cand - q);
    add += (uint64_t)(sv < 0 ? -(int64_t)sv : (int64_t)sv);
    found++;
    if constexpr (CX::emit) {
      uint64_t v = fixed | (1ull << (cand - q));
      if (ridge >= 0) v |= 1ull << (ridge - q);
      emit_cell(cx, v);
    }
  }
  if (lane_id() == 0) {
    cx.tally->acc += add;
    cx.tally->cells += found;
    if (zero) cx.tally->tie = 1;
  }
}

// Leaves of one ridge whose state is identical in every group: the groups
// test consecutive candidates c, c-1, ... of the ridge in one step.
template <class CX>
__device__ __forceinline__ void leaves_uniform(CX &cx, const St<1> &st, int hi_c, int lo_c) {
  const int G = cx.G();
  const int32_t sig = st.s[0], H1 = st.H1, H0 = st.H0;
  const bool prevneg = st.prev < 0;
  const uint64_t excl = ~cx.valid_lanes | cx.chosen_rep;
  const uint64_t fixed = CX::emit ? (cx.chosen_rep & group0_mask(cx)) : 0ull;
  if (hi_c < lo_c) return;
  if constexpr (CX::single) {
    // one group: visit only the candidates with D = sigma_c != 0 (the chosen
    // points have a zero residual and drop out by themselves)
    const uint64_t range = ((2ull << hi_c) - 1) & ~((1ull << lo_c) - 1);
    uint64_t todo = ballot(sig != 0) & cx.valid_lanes & range;
    if (!charge(cx, __builtin_popcountll(todo))) return;
    while (todo) {
      const int c0 = __builtin_ctzll(todo); // any order: the tallies are sums
      todo &= ~(1ull << c0);
      // t' = s (sigma_c h_j - h_c sigma_j) with s the (wave-uniform) sign of
      // D prev, folded into the candidate's scalar values: a = s sigma_c and
      // -b = -s h_c (|sigma_c| < 2^31, so the negations are exact)
      const int32_t sc = rl32(sig, c0), h1c = rl32(H1, c0), h0c = rl32(H0, c0);
      const bool flip = (sc < 0) != prevneg;
      const Cross t = cross_view(flip ? -sc : sc, flip ? h1c : -h1c, flip ? h0c : -h0c, sig, H1, H0);
      decide(cx, ballot(t.C < 0), t, cx.top_bits, excl, sig, c0, fixed, -1);
    }
    return;
  }
  if (!charge(cx, (hi_c - lo_c + G) / G)) return;
  const View v = cand_view(sig, H1, H0, prevneg);
  for (int c0 = hi_c; c0 >= lo_c; c0 -= G) {
    const int cg = c0 - cx.g;
    const bool ok = cg >= lo_c;
    const int src = cx.g * cx.npad() + (ok ? cg : 0);
    const int32_t a = fetch_diag(cx, v.a, c0, src);
    const Cross t = cross_view(a, fetch_diag(cx, v.nb1, c0, src), fetch_diag(cx, v.nb0, c0, src), sig, H1, H0);
    decide(cx, ballot(t.C < 0), t, ballot(ok) & ballot(a != 0) & cx.top_bits, excl, sig, c0, fixed,
           -1);
  }
}

// Range of the next element at depth T (T+1 points chosen, lowest `low`).
template <class CX>
__device__ __forceinline__ bool next_range(const CX &cx, int T, int K, int low, int *hi_c, int *lo_c) {
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
template <int K, int T, class CX>
struct Level {
  static __device__ __forceinline__ void run(CX &cx, const St<K - T> &st, int low) {
    constexpr bool S = CX::stats;
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
        Level<K, T + 1, CX>::run(cx, ch, c);
        cx.chosen_rep &= ~(cx.rep_unit << c);
      }
    } else {
      // T = k-2: create ridges (depth k-1) from a 2-column state, then test
      // their candidates.
      static_assert(W == 2, "ridge level");
      const Div dv = make_div(st.prev);
      if (forced || CX::single || cx.G() == 1) {
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
          if constexpr (S) {
            cx.ridges++;
            cx.rsteps++;
          }
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
        const int G = cx.G();
        for (int c = hi_c; c >= lo_c && step_ok(cx); c -= G) {
          const int cg = c - cx.g;
          const bool gok = cg >= lo_c;
          const int src = cx.g * cx.npad() + (gok ? cg : 0);
          const int32_t r0 = bp32(st.s[0], src), r1 = bp32(st.s[1], src);
          const int32_t h1c = bp32(st.H1, src), h0c = bp32(st.H0, src);
          const bool p0 = r0 != 0;
          const int32_t piv = p0 ? r0 : (r1 != 0 ? r1 : 1);
          const int32_t rco = p0 ? r1 : r0;
          const int32_t rjp = p0 ? st.s[0] : st.s[1], so = p0 ? st.s[1] : st.s[0];
          const int32_t sig = exdiv32((int64_t)piv * so - (int64_t)rco * rjp, dv);
          const int64_t A = (int64_t)piv * st.H1 - (int64_t)h1c * rjp;
          const int64_t B = (int64_t)piv * st.H0 - (int64_t)h0c * rjp;
          const int64_t h = exdiv_split(A, B, dv);
          const int32_t H1 = (int32_t)(h >> 31), H0 = (int32_t)((uint32_t)h & LOW31);
          const bool pivneg = piv < 0;
          // (ballots of single compares, ANDed in scalar registers)
          const uint64_t m_alive = ballot(gok) & ballot((r0 | r1) != 0);
          const int ngr = min(G, c - lo_c + 1);
          if constexpr (S) {
            const uint32_t n_alive = (uint32_t)__builtin_popcountll(m_alive & cx.rep_unit);
            cx.ridges += n_alive;
            cx.pruned += (uint32_t)ngr - n_alive;
            cx.rsteps++;
          }
          if (!m_alive) continue;
          const uint64_t alive_top = m_alive & cx.top_bits;
          const uint64_t excl = ~cx.valid_lanes | cx.chosen_rep | diag_lanes(cx, c);
          const uint64_t fixed = CX::emit ? (cx.chosen_rep & group0_mask(cx)) : 0ull;
          // candidates: group q tests cc - q for cc = c-1 .. 0, visiting only
          // the cc for which some live group's point cc - q has D != 0 (lane
          // j of group q stands for cc = j + q; chosen and ridge points have
          // a zero residual and drop out by themselves)
          const uint64_t nzl = m_alive & ballot(sig != 0) & cx.valid_lanes;
          const View v = cand_view(sig, H1, H0, pivneg);
          const int base = cx.g * cx.npad() - cx.g; // lane of point cc - g is base + cc
          const int npl = cx.npl();
          const uint64_t gm0 = (1ull << cx.npad()) - 1;
          uint64_t todo = 0;
          if (G == 2) // the common case (17 to 32 points), without a loop
            todo = (nzl & gm0) | ((nzl >> 32) << 1);
          else
            for (int q = 0; q < G; q++) todo |= ((nzl >> (q << npl)) & gm0) << q;
          todo &= (1ull << c) - 1;
          if (!charge(cx, __builtin_popcountll(todo))) continue;
          while (todo) {
            const int cc = __builtin_ctzll(todo); // any order: the tallies are sums
            todo &= ~(1ull << cc);
            // cc < g: no candidate in group g (the fetch reads a lane of the
            // group below, in range, and is masked out of `has`)
            const int src2 = base + cc;
            const int32_t a = bp32(v.a, src2);
            const Cross t = cross_view(a, bp32(v.nb1, src2), bp32(v.nb0, src2), sig, H1, H0);
            // (two ballots: a ballot of the combined condition would go through a VGPR)
            const uint64_t has = ballot(a != 0) & ballot(cc >= cx.g) & alive_top;
            decide(cx, ballot(t.C < 0), t, has, excl, sig, cc, fixed, c);
          }
        }
      }
    }
  }
};

template <int K, class CX>
__device__ __forceinline__ void process_tile(CX &cx, const SysDesc &sd, const int32_t *__restrict__ pts,
                                             const int64_t *__restrict__ hts) {
  constexpr bool S = CX::stats;
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
  // padding lanes start from a zero row: every residual derived from it (a
  // combination of the lane's own entries) stays exactly zero, so their t'
  // is 0 and the strict test never needs to mask them
  const int64_t h0 = valid ? w - wb : 0;
  St<K> st;
#pragma unroll
  for (int i = 0; i < K; i++) st.s[i] = valid ? P[i] - rl32(P[i], base) : 0;
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
    Level<K, 0, CX>::run(cx, st, base);
  }
}

// One work unit.
template <int KLO, int KHI, int MODE, int GG>
__device__ __forceinline__ void run_unit(const Tile &tl, const SysDesc &sd, const int32_t *__restrict__ pts,
                                         const int64_t *__restrict__ hts, SysAcc *__restrict__ acc,
                                         DevCounters *__restrict__ cnt, const CellSink &sink, Tally *tally) {
  using CX = Ctx<MODE, GG>;
  constexpr bool S = CX::stats;
  const int lane = lane_id();
  CX cx;
  cx.npl_ = sd.npad_log2;
  cx.G_ = 64 >> sd.npad_log2;
  cx.g = lane >> cx.npl();
  cx.j = lane & (cx.npad() - 1);
  cx.jg = cx.j + cx.g;
  cx.mask = tl.mask;
  cx.L = __builtin_popcountll(tl.mask);
  cx.c_lo = tl.c_lo;
  cx.c_hi = tl.c_hi;
  uint64_t unit = 0, vl = 0, top = 0;
  const uint64_t pm = sd.N >= 64 ? ~0ull : ((1ull << sd.N) - 1);
  for (int q = 0; q < cx.G(); q++) {
    unit |= 1ull << (q * cx.npad());
    top |= 1ull << (q * cx.npad() + cx.npad() - 1);
    vl |= pm << (q * cx.npad());
  }
  cx.rep_unit = unit;
  cx.top_bits = top;
  cx.valid_lanes = vl;
  cx.tally = tally;
  if (lane == 0) {
    tally->acc = 0;
    tally->cells = 0;
    tally->tie = 0;
  }
  cx.leaves = cx.ridges = cx.inner = cx.sp_upd = cx.pruned = cx.rsteps = cx.lsteps = cx.lempty = 0;
  cx.sink = sink;
  {
    // every loop step of a unit is charged to a candidate below it, and a
    // candidate is charged at most once per depth: k + 1 steps suffice
    const uint64_t cand = unit_candidates(sd.k, tl.mask, tl.c_lo, tl.c_hi);
    const uint64_t b = cand * (uint64_t)(sd.k + 3) + 256;
    cx.left = b > 0x7FFFFFF0ull ? 0x7FFFFFF0 : (int32_t)b;
  }
  switch (sd.k) {
#define BDEG_CASE(KK)                                      \
  case KK:                                                 \
    if constexpr (KK >= KLO && KK <= KHI)                  \
      process_tile<KK, CX>(cx, sd, pts, hts);              \
    break;
    BDEG_CASE(1) BDEG_CASE(2) BDEG_CASE(3) BDEG_CASE(4) BDEG_CASE(5) BDEG_CASE(6)
    BDEG_CASE(7) BDEG_CASE(8) BDEG_CASE(9) BDEG_CASE(10) BDEG_CASE(11) BDEG_CASE(12)
    BDEG_CASE(13) BDEG_CASE(14) BDEG_CASE(15) BDEG_CASE(16) BDEG_CASE(17) BDEG_CASE(18)
#undef BDEG_CASE
    default:
      break;
  }
  const bool abandoned = cx.left <= 0;
  if (lane == 0 && abandoned) atomicOr(&cnt->error, 1u);
  if (lane == 0 && !abandoned) {
    const unsigned long long sum = tally->acc;
    const uint32_t cells = tally->cells, tie = tally->tie;
    if (sum | cells | tie) {
      SysAcc *a = &acc[tl.sys];
      const unsigned long long old = atomicAdd((unsigned long long *)&a->lo, sum);
      if (old + sum < old) atomicAdd((unsigned long long *)&a->hi, 1ull);
      atomicAdd((unsigned long long *)&a->cells, (unsigned long long)cells);
      if (tie) atomicOr(&a->tie, 1u);
    }
    if constexpr (S) {
      atomicAdd((unsigned long long *)&cnt->ridges, (unsigned long long)cx.ridges);
      atomicAdd((unsigned long long *)&cnt->inner, (unsigned long long)cx.inner);
      atomicAdd((unsigned long long *)&cnt->sp_upd, (unsigned long long)cx.sp_upd);
      atomicAdd((unsigned long long *)&cnt->leaves, (unsigned long long)cx.leaves);
      atomicAdd((unsigned long long *)&cnt->rsteps, (unsigned long long)cx.rsteps);
      atomicAdd((unsigned long long *)&cnt->lsteps, (unsigned long long)cx.lsteps);
      atomicAdd((unsigned long long *)&cnt->lempty, (unsigned long long)cx.lempty);
      atomicAdd((unsigned long long *)&cnt->pruned, (unsigned long long)cx.pruned);
      atomicAdd((unsigned long long *)&cnt->tiles, 1ull);
      // a unit belongs to one system, so weighting its counts by that
      // system's point count is exact for batches of mixed N and k
      const unsigned long long n = (unsigned long long)sd.N, t = (unsigned long long)(sd.N - sd.k - 1);
      atomicAdd((unsigned long long *)&cnt->w_inner, n * cx.inner);
      atomicAdd((unsigned long long *)&cnt->w_spatial, n * cx.sp_upd);
      atomicAdd((unsigned long long *)&cnt->w_ridges, n * cx.ridges);
      atomicAdd((unsigned long long *)&cnt->w_leaves, t * cx.leaves);
    }
  }
}

// Waves per SIMD each depth is compiled for: the register budget grows with k
// (one residual row per level), so deeper kernels trade occupancy for no
// spills.  The single-group variant needs fewer registers (no sibling-ridge
// path): at k = 10 it fits five waves.
constexpr int waves_for_depth(int k, int gg) {
  return k <= 3 ? 8 : k <= 7 ? 7 : k == 8 ? 6 : k == 9 ? 5 : k == 10 ? (gg == 1 ? 5 : 4) : k == 11 ? 4 : k <= 14 ? 3 : 2;
}

template <int KLO, int KHI, int MODE, int GG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_for_depth(KHI, GG))))
enum_kernel(const SysDesc *__restrict__ sys, const int32_t *__restrict__ pts, const int64_t *__restrict__ hts,
            const Tile *__restrict__ tiles, uint32_t n_tiles, SysAcc *__restrict__ acc,
            DevCounters *__restrict__ cnt, CellSink sink, const uint32_t *__restrict__ rerun) {
  const int lane = lane_id();
  __shared__ Tally tallies[4]; // one per wavefront of the block (at most 256 threads)
  Tally *tally = &tallies[threadIdx.x >> 6];
  // an in-pass redraw round with nothing to redraw ends at once (uniform load)
  if (rerun && rerun[0] == 0) return;
  for (;;) {
    // Every lane takes part in the claim (lane 0 adds one, the others zero)
    // and lane 0's result is read by index, so the claimed unit is uniform by
    // construction and no lane-dependent branch surrounds the loop's exit
    // test (with a lane-0 branch the compiler may split the loop so that
    // lanes 1..63 wait for a value lane 0 never produces).
    const uint32_t claim = atomicAdd(&cnt->next_tile, lane == 0 ? 1u : 0u);
    const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int32_t)claim, 0);
    if (t >= n_tiles) break;
    const Tile tl = tiles[t];
    if (rerun && rerun[1 + tl.sys] == 0) continue; // this system's sums stand
    const SysDesc sd = sys[tl.sys];
    run_unit<KLO, KHI, MODE, GG>(tl, sd, pts, hts, acc, cnt, sink, tally);
  }
}

} // namespace dev


} // namespace bdeg

// Instantiation helper: one translation unit per k range defines
// bdeg::enum_fn_<klo>_<khi>(mode, single).  The emitting variant exists for
// single-k kernels only.
namespace bdeg {
namespace dev {
template <int KLO, int KHI, int MODE>
EnumFn pick_variant(bool single) {
  if (single) return enum_kernel<KLO, KHI, MODE, 1>;
  return enum_kernel<KLO, KHI, MODE, 0>;
}
template <int KLO, int KHI>
EnumFn pick_kernel(int mode, bool single) {
  if (mode == MODE_STATS) return pick_variant<KLO, KHI, MODE_STATS>(single);
  if (mode == MODE_EMIT) {
    if constexpr (KLO == KHI) return pick_variant<KLO, KHI, MODE_EMIT>(single);
    else return nullptr;
  }
  return pick_variant<KLO, KHI, MODE_PLAIN>(single);
}
} // namespace dev
} // namespace bdeg

