// Device code of the lane-dense enumeration kernel (included by the per-k
// translation units, which instantiate it next to enum_device.hpp's kernel).
#pragma once
// What is computed is the same as in enum_device.hpp (Section 4, eqs.
// "lower-face" and "simplex-vol", strict as in eq. "lower-d-face-again"):
// for every candidate (k+1)-subset of the lifted points, whether every other
// lifted point lies strictly above the hyperplane through it, and then
// |det| of its spatial differences.  Only the schedule differs.
//
//   * A wavefront walks a work unit's subtree depth-first with lane j holding
//     point j (one fraction-free Bareiss step per chosen point, as in
//     enum_device.hpp), but stops with three spatial columns left: at a node
//     with k - 2 points chosen, lane j holds (s0, s1, s2, h) of point j, the
//     (T+1)-minors of the chosen difference rows bordered by point j.
//   * The node's candidates are its triples {c1 > c2 > c3} below the lowest
//     chosen point.  Lanes now stand for triples: each derives, from the
//     node's rows c1, c2, c3 (in LDS), the triple's exact cofactors by
//     Sylvester's identity -- the k x k spatial minor D and three height
//     minors -- so that for every point j
//         u_j = -s0_j H0 + s1_j H1 - s2_j H2 + h_j D = prev * M_j,
//     where M_j is the (k+1)-minor of the candidate's rows and point j's row
//     (point j's height over the candidate's hyperplane, times D) and prev is
//     the node's last pivot.  A candidate is a lower facet exactly when
//     sign(D) sign(prev) u_j > 0 for every point j off the candidate.
//   * Triples with D != 0 go into a ring of records in LDS; a test batch
//     takes 64 records and loops over the points, every lane testing its own
//     candidate against point j (row j is one broadcast LDS read), so all 64
//     lanes do the same useful work and consecutive points are independent
//     chains.  The test is four 32 x 32 -> 64 multiply-adds per point: exact
//     when the record's coefficients and the node's heights fit 31 and 32
//     bits; otherwise both are shifted right by one amount and the sum,
//     with a bound on what the shift dropped, proves a point below or leaves
//     the candidate to the exact decision.
//   * The three most recent nodes keep their rows in three LDS tables, so a
//     setup pass or a test batch may hold candidates of all of them: passes
//     and batches stay full although most nodes have only a few candidates
//     (a node whose lowest chosen point is c has C(c, 3)).  A node is
//     finished only when a new node needs its table; that drains the
//     pipeline (a last batch of fewer than 64 records splits each
//     candidate's points over several lanes), and the next two new nodes
//     then find their tables free.  The pipeline also runs on across the
//     work units of one system; a change of system, or the end, drains it.
//   * The rare candidates with no point proved below are decided exactly
//     with lanes as points: a point strictly below rejects, and the zero
//     count tells a lower facet (exactly the k + 1 vertices vanish) from a
//     tie.
//
// Widths (certified on the host for these systems: spatial minors < 2^30,
// height minors < 2^59): the cofactors are formed with heights and height
// minors split as x = xh 2^29 + xl, 0 <= xl < 2^29, so every product is a
// 32 x 32 -> 64 multiply-add; the exact decision sums u_j the same way (low
// limbs below 2^61, high limbs below 2^62; u_j < 0 exactly when its high
// part, with the low part's carry, is negative).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"
#include "enum_device.hpp"
#include "exact_div.hpp"

namespace bdeg {
namespace dev {

constexpr int DENSE_LIMB = 29;
constexpr int64_t DENSE_LMASK = (1ll << DENSE_LIMB) - 1;
constexpr int DENSE_RING = 128; // candidate records per wavefront (a power of two >= 2 * 64)
constexpr int DENSE_TABLES = 3; // row tables: the most recent nodes in flight
constexpr int DENSE_TAIL = 7;   // children below this point: quadruples set up from their parent

// What the setup passes and the exact decisions need of the node in a row
// table (kept in LDS, not in scalar registers).
struct TableInfo {
  uint64_t inv;    // the 2-adic inverse of the node's pivot (sign folded in)
  uint64_t chosen; // its chosen points (vertices shared by its candidates)
  uint32_t e;      // the pivot's 2-adic valuation
  uint32_t prevneg; // pivot < 0
  uint32_t sig;    // the table holds h >> sig, which fits int32
  uint32_t band;   // the largest |s0| + |s1| + |s2| of its points (BAND_UNSET: not needed yet)
};
constexpr uint32_t BAND_UNSET = 0xFFFFFFFFu;

// Per-wavefront LDS: the point rows of the most recent nodes and the record
// ring.
struct alignas(16) DenseLds {
  int4 rowS[DENSE_TABLES][64];            // s0, s1, s2, h >> sig
  int2 rowH[DENSE_TABLES][64];            // h split at bit 29: hh, hl
  int4 recX[DENSE_RING];    // a candidate's filter coefficients k0 >> sg, k1 >> sg, k2 >> sg and d
  int32_t recM[DENSE_RING]; // c1 | c2 << 8 | c3 << 16 | table | shift sg
  TableInfo info[DENSE_TABLES];
  uint8_t perm[64]; // lane j holds point perm[j] of the system (its lifted-height order, or j)
  // rows of the node whose tail quadruples are set up (four spatial columns)
  int4 qS[64];  // s0, s1, s2, s3
  int32_t qh[64]; // h >> its shift
  int2 qx[8];   // h split at bit 29 (hh, hl) of the points below DENSE_TAIL
  // rows of the tail's children (child c0, point x < c0 at C(c0,2) - 3 + x)
  int4 ctS[18];
  int2 ctH[18];
  Tally tally;
};
// four blocks of four waves fit a compute unit's 160 KiB
static_assert(16 * sizeof(DenseLds) <= 160 * 1024, "lane-dense LDS limits occupancy below four waves per SIMD");

// One node held in a row table (wave-uniform values).
struct NodeInfo {
  int t;               // its row table (and TableInfo)
  uint32_t r_cur, r_hi; // its triples still to set up: colex ranks [r_cur, r_hi)
  uint32_t recs;       // its records in the ring
};

template <int MODE>
struct DCtx {
  static constexpr bool stats = MODE == MODE_STATS;
  static constexpr bool emit = MODE == MODE_EMIT;
  int N, k, j;
  uint64_t mask;   // work unit prefix
  int L;           // prefix length
  int c_lo, c_hi;  // sibling run at the first free level
  uint64_t chosen; // chosen points of the current depth-first node
  DenseLds *lds;
  // The most recent nodes, oldest first (each in its own row table).  A
  // setup pass takes the oldest node's triples first, then the next ones';
  // the record ring is in the same order.  (Indexed by constants only, so
  // that they stay in scalar registers.)
  NodeInfo nd[DENSE_TABLES];
  int head, nrec;  // record ring: first record and count (wave-uniform)
  int32_t left;    // watchdog budget (as in enum_device.hpp)
  uint32_t inner, sp_upd, pruned, nodes, triples, leaves, setups, tests, wide, quads;
  uint32_t lpts; // per lane: points examined by its candidates' tests (counting variant)
  CellSink sink;
};

__device__ __forceinline__ void wave_sync_lds() {
  // LDS written by some lanes is read by others of the same wavefront
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (Hi 2^29 + Lo) / d for an exact multiple whose quotient fits int64 (e <= 29).
__device__ __forceinline__ int64_t exdiv_limbs(int64_t Hi, int64_t Lo, const Div &d) {
  const uint64_t y = ((uint64_t)Hi << (DENSE_LIMB - d.e)) + (uint64_t)(Lo >> d.e);
  return (int64_t)(y * d.inv);
}

// Colex unranking of a 3-subset {c1 > c2 > c3}: rank = C(c1,3) + C(c2,2) + c3.
// Compares 6 r with c (c-1) (c-2) (no division); r < C(64, 3).  No bound
// tests are needed: c1 = 64 (or 65) already fails, as 6 r < 64 * 63 * 62,
// and c2 >= c1 fails, as the remainder is below C(c1, 2); so each step is a
// compare and a select.
__device__ __forceinline__ void unrank3(uint32_t r, int *c1, int *c2, int *c3) {
  const uint32_t r6 = 6u * r;
  uint32_t a = 2;
#pragma unroll
  for (uint32_t step = 32; step >= 1; step >>= 1) {
    const uint32_t x = a + step;
    a = __umul24(__umul24(x, x - 1), x - 2) <= r6 ? x : a;
  }
  const uint32_t rem2 = (r6 - __umul24(__umul24(a, a - 1), a - 2)) / 3u; // 2 (C(c2,2) + c3)
  uint32_t b = 1;
#pragma unroll
  for (uint32_t step = 32; step >= 1; step >>= 1) {
    const uint32_t x = b + step;
    b = __umul24(x, x - 1) <= rem2 ? x : b;
  }
  *c1 = (int)a;
  *c2 = (int)b;
  *c3 = (int)((rem2 - __umul24(b, b - 1)) >> 1);
}

__device__ __forceinline__ uint32_t c3_of(int c) { return (uint32_t)(c * (c - 1) * (c - 2) / 6); }
__device__ __forceinline__ uint32_t c2_of(int c) { return (uint32_t)(c * (c - 1) / 2); }

// a * M into the limb sums (M = Mh 2^29 + Ml, |a| < 2^30, |M| < 2^59)
__device__ __forceinline__ void acc_limbs(int64_t &Hi, int64_t &Lo, int32_t a, int64_t M) {
  Hi += (int64_t)a * (int32_t)(M >> DENSE_LIMB);
  Lo += (int64_t)a * (int32_t)(M & DENSE_LMASK);
}

// A candidate record holds what its filter test needs: k_a >> sg (a = 0, 1,
// 2) and d, and a word with c1 | c2 << 8 | c3 << 16, its node table in the
// two bits at REC_TABLE_BIT and the shift sg in the five bits at
// REC_SHIFT_BIT.  The exact cofactors of the rare candidates the filter
// cannot reject are derived again from the table.
constexpr int REC_TABLE_BIT = 25;
constexpr int REC_SHIFT_BIT = 27;

// Wave-wide sum (every lane active), as wave_umax below.
__device__ __forceinline__ uint32_t wave_usum(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false); // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false); // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false); // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false); // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false); // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false); // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Wave-wide maximum of an unsigned value (every lane active): a row-wise DPP
// shift scan, then the row broadcasts; lane 63 ends with the maximum.
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false)); // row_shr:1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false)); // row_shr:2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false)); // row_shr:4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false)); // row_shr:8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false)); // row_bcast:15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false)); // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}



// A vertex set in the system's own point labels (lane j holds point perm[j]).
template <class CX>
__device__ __forceinline__ uint64_t unlabel(const CX &cx, uint64_t verts) {
  uint64_t m = 0;
  while (verts) {
    const int b = __builtin_ctzll(verts);
    verts &= verts - 1;
    m |= 1ull << cx.lds->perm[b];
  }
  return m;
}

// The lane order of a system's points: when its units cover all its
// candidates (SYS_SORTED) the kernel relabels the points in ascending lifted
// height (ties by index), which changes no candidate's decision but lets a
// test batch, which walks the points in label order, meet a point below each
// candidate sooner; otherwise the identity.  Called by every lane.
template <class CX>
__device__ __forceinline__ void dense_order(CX &cx, const SysDesc &sd, const int64_t *__restrict__ hts) {
  const int lane = lane_id();
  int rank = lane;
  if (sd.flags & SYS_SORTED) {
    const int64_t h = lane < sd.N ? hts[sd.ht_off + lane] : INT64_MAX;
    rank = 0;
    for (int i = 0; i < 64; i++) {
      const int64_t hi = (int64_t)(((uint64_t)(uint32_t)rl32((int32_t)((uint64_t)h >> 32), i) << 32) |
                                   (uint32_t)rl32((int32_t)(uint32_t)(uint64_t)h, i));
      rank += (hi < h || (hi == h && i < lane)) ? 1 : 0;
    }
  }
  wave_sync_lds();
  cx.lds->perm[rank] = (uint8_t)lane;
  wave_sync_lds();
}

// Cofactors of the triple {c1 > c2 > c3} of a node, from its rows (RS:
// s0, s1, s2; RH: heights split at bit 29: h = hh 2^29 + l, 0 <= l < 2^29) and its
// pivot data: the 2 x 2 minors of rows c1, c2 (T+2 minors), spatial and
// with the height column; then the 3 x 3 minors of rows c1, c2, c3 (T+3
// minors) by expansion along row c3: the spatial one D first, then, with
// row c3 multiplied by the orientation sign(D) sign(prev) (every minor
// below is linear in it), the coefficients of u_j: k0 = -H0, k1 = H1,
// k2 = -H2 (H_a: column a deleted); d is D times the same sign.
__device__ __forceinline__ void triple_cofactors(const int4 *RS, const int2 *RH, int c1, int c2, int c3, const Div &dv,
                                                 bool prevneg, int64_t &k0, int64_t &k1, int64_t &k2, int32_t &D,
                                                 int32_t &d) {
  const int4 a1 = RS[c1], a2 = RS[c2], a3 = RS[c3];
  const int2 x1 = RH[c1], x2 = RH[c2], x3 = RH[c3];
  const int32_t hh1 = x1.x, l1 = x1.y, hh2 = x2.x, l2 = x2.y, hh3 = x3.x, l3 = x3.y;
  const int32_t s01 = a1.x, s11 = a1.y, s21 = a1.z;
  const int32_t s02 = a2.x, s12 = a2.y, s22 = a2.z;
  const int32_t s03 = a3.x, s13 = a3.y, s23 = a3.z;
  const int32_t m01 = exdiv32((int64_t)s01 * s12 - (int64_t)s11 * s02, dv);
  const int32_t m02 = exdiv32((int64_t)s01 * s22 - (int64_t)s21 * s02, dv);
  const int32_t m12 = exdiv32((int64_t)s11 * s22 - (int64_t)s21 * s12, dv);
  const int64_t m0h = exdiv_limbs((int64_t)s01 * hh2 - (int64_t)hh1 * s02, (int64_t)s01 * l2 - (int64_t)l1 * s02, dv);
  const int64_t m1h = exdiv_limbs((int64_t)s11 * hh2 - (int64_t)hh1 * s12, (int64_t)s11 * l2 - (int64_t)l1 * s12, dv);
  const int64_t m2h = exdiv_limbs((int64_t)s21 * hh2 - (int64_t)hh1 * s22, (int64_t)s21 * l2 - (int64_t)l1 * s22, dv);
  D = exdiv32((int64_t)s03 * m12 - (int64_t)s13 * m02 + (int64_t)s23 * m01, dv);
  const bool flip = (D < 0) != prevneg;
  const int32_t P0 = flip ? -s03 : s03, P1 = flip ? -s13 : s13, P2 = flip ? -s23 : s23;
  const int32_t Ph = flip ? -hh3 : hh3, Pl = flip ? -l3 : l3;
  int64_t Hi, Lo;
  Hi = (int64_t)(-Ph) * m12, Lo = (int64_t)(-Pl) * m12;
  acc_limbs(Hi, Lo, -P1, m2h);
  acc_limbs(Hi, Lo, P2, m1h);
  k0 = exdiv_limbs(Hi, Lo, dv); // -H0, columns s1, s2, h
  Hi = (int64_t)Ph * m02, Lo = (int64_t)Pl * m02;
  acc_limbs(Hi, Lo, P0, m2h);
  acc_limbs(Hi, Lo, -P2, m0h);
  k1 = exdiv_limbs(Hi, Lo, dv); // H1, columns s0, s2, h
  Hi = (int64_t)(-Ph) * m01, Lo = (int64_t)(-Pl) * m01;
  acc_limbs(Hi, Lo, -P0, m1h);
  acc_limbs(Hi, Lo, P1, m0h);
  k2 = exdiv_limbs(Hi, Lo, dv); // -H2, columns s0, s1, h
  d = flip ? -D : D;
}

// Exact decision of one candidate (its record word, wave-uniform) that the
// filter could not reject, with lanes as points: its cofactors derived
// again, u_j = k0 s0 + k1 s1 + k2 s2 + d h summed in limbs as
// u = 2^29 hi + (lo mod 2^29) (every product a 32 x 32 -> 64 multiply-add;
// the low limbs sum below 2^61, the high limbs below 2^62).  Rejected when
// a point lies strictly below; a lower facet when exactly its k + 1
// vertices vanish; a tie otherwise.
template <class CX>
__device__ __forceinline__ void decide_exact(CX &cx, int32_t meta) {
  const int lane = lane_id();
  const int t = (meta >> REC_TABLE_BIT) & 3;
  const int c1 = meta & 255, c2 = (meta >> 8) & 255, c3 = (meta >> 16) & 255;
  const TableInfo ti = cx.lds->info[t];
  Div dv;
  dv.e = ti.e;
  dv.inv = ti.inv;
  int64_t k0, k1, k2;
  int32_t D, d;
  triple_cofactors(cx.lds->rowS[t], cx.lds->rowH[t], c1, c2, c3, dv, ti.prevneg != 0, k0, k1, k2, D, d);
  const int4 row = cx.lds->rowS[t][lane];
  const int2 hx = cx.lds->rowH[t][lane];
  const int64_t lo = (int64_t)row.x * (int32_t)(k0 & DENSE_LMASK) + (int64_t)row.y * (int32_t)(k1 & DENSE_LMASK) +
                     (int64_t)row.z * (int32_t)(k2 & DENSE_LMASK) + (int64_t)hx.y * d;
  const int64_t hi = (lo >> DENSE_LIMB) + (int64_t)row.x * (int32_t)(k0 >> DENSE_LIMB) +
                     (int64_t)row.y * (int32_t)(k1 >> DENSE_LIMB) + (int64_t)row.z * (int32_t)(k2 >> DENSE_LIMB) +
                     (int64_t)hx.x * d;
  const bool on = hi == 0 && (lo & DENSE_LMASK) == 0;
  const uint64_t zero = ballot(on && lane < cx.N);
  const uint64_t below = ballot(hi < 0 && lane < cx.N);
  if (below) return; // a point below within the filter's band
  const uint64_t verts = ti.chosen | (1ull << c1) | (1ull << c2) | (1ull << c3);
  if (zero != verts) {
    if (lane == 0) cx.lds->tally.tie = 1;
    return;
  }
  if (lane == 0) {
    cx.lds->tally.acc += (unsigned long long)(d < 0 ? -(int64_t)d : (int64_t)d);
    cx.lds->tally.cells += 1;
  }
  if constexpr (CX::emit) emit_cell(cx, unlabel(cx, verts));
}

// The points of a full test batch (one candidate per lane) until every
// valid lane has a point proved below (neg < 0), checked every four points.
// (The counting variant also records, per lane, how many points its
// candidate needed: up to its first point proved below.)
template <bool SHIFT, bool STATS>
__device__ __forceinline__ void test_points_early(const int4 *rowS, int iters, bool valid, int32_t x0, int32_t x1,
                                                  int32_t x2, int32_t d, int64_t bnd, int dl, int32_t &neg,
                                                  int32_t &first) {
#pragma unroll 4
  for (int j = 0; j < iters; j++) {
    const int4 r = rowS[j];
    const int32_t hj = SHIFT ? (r.w >> dl) : r.w;
    const int64_t v = bnd + (int64_t)r.x * x0 + (int64_t)r.y * x1 + (int64_t)r.z * x2 + (int64_t)hj * d;
    neg |= (int32_t)((uint64_t)v >> 32);
    if constexpr (STATS)
      if (first == 0 && neg < 0) first = j + 1;
    if ((j & 3) == 3 && ballot(valid && neg >= 0) == 0) break;
  }
}

// Test the n oldest records of the ring (n <= 64), each over all points, its
// points split over 2^logC lanes.
template <class CX>
__device__ __forceinline__ void test_batch(CX &cx, int n, int logC) {
  const int lane = lane_id();
  const int p = lane >> logC, q = lane & ((1 << logC) - 1);
  const bool valid = p < n;
  const int slot = (cx.head + (valid ? p : 0)) & (DENSE_RING - 1);
  const int4 rx = cx.lds->recX[slot];
  const int32_t meta = cx.lds->recM[slot];
  // Filter test, exact in its rejections.  A record's shift sg makes its
  // coefficients k_a >> sg fit 31 bits and its node's heights h >> sg fit 32
  // (the row table holds h >> sn, sn <= sg; a lane shifts on by sg - sn).
  // Then u_j = 2^sg v_j + e_j, v_j = sum_a (k_a >> sg) s_aj + d (h_j >> sg),
  // with 0 <= the dropped low parts < 2^sg, so |e_j| < 2^sg (|s0| + |s1| +
  // |s2| + |d|) and v_j + B + |d| <= 0 (B: the node's largest |s0| + |s1| +
  // |s2|) proves u_j < 0.  With sg = 0 (coefficients and heights fit, the
  // common case for 20-bit liftings) v_j is u_j and the test is exact.
  // Every sum is four products below 2^61 plus the band: below 2^63.  A
  // candidate with a point proved below is rejected; one without is decided
  // exactly below.
  const int iters = (cx.N + (1 << logC) - 1) >> logC; // rows past N are zero rows
  const int t = (meta >> REC_TABLE_BIT) & 3;
  const int sg = (int)((uint32_t)meta >> REC_SHIFT_BIT);
  const uint2 sb = *(const uint2 *)&cx.lds->info[t].sig; // (sig, band) of the record's table
  const int dl = sg - (int)sb.x;
  const int32_t x0 = rx.x, x1 = rx.y, x2 = rx.z, d = rx.w;
  const int64_t bnd = sg > 0 ? (int64_t)sb.y + (d < 0 ? -(int64_t)d : (int64_t)d) - 1 : 0;
  const int4 *rowS = cx.lds->rowS[t];
  int32_t neg = 0, first = 0;
  const bool shifted = ballot(valid && dl != 0) != 0;
  if (logC == 0) {
    // a full batch stops once every candidate has a point proved below
    if (!shifted)
      test_points_early<false, CX::stats>(rowS, iters, valid, x0, x1, x2, d, bnd, 0, neg, first);
    else
      test_points_early<true, CX::stats>(rowS, iters, valid, x0, x1, x2, d, bnd, dl, neg, first);
  } else if (!shifted) {
#pragma unroll 4
    for (int it = 0; it < iters; it++) {
      const int j = q + (it << logC); // < 64: 2^logC divides 64 and N <= 64
      const int4 r = rowS[j];
      const int64_t v = bnd + (int64_t)r.x * x0 + (int64_t)r.y * x1 + (int64_t)r.z * x2 + (int64_t)r.w * d;
      neg |= (int32_t)((uint64_t)v >> 32);
    }
  } else {
#pragma unroll 4
    for (int it = 0; it < iters; it++) {
      const int j = q + (it << logC);
      const int4 r = rowS[j];
      const int64_t v = bnd + (int64_t)r.x * x0 + (int64_t)r.y * x1 + (int64_t)r.z * x2 + (int64_t)(r.w >> dl) * d;
      neg |= (int32_t)((uint64_t)v >> 32);
    }
  }
  if constexpr (CX::stats) {
    cx.tests++;
    // points examined: up to the first point proved below (full batches),
    // else every other point
    if (valid && q == 0) cx.lpts += (uint32_t)((logC == 0 && first > 0) ? first : cx.N - cx.k - 1);
  }
  const uint64_t rej = ballot(neg < 0);
  const int C = 1 << logC;
  const uint64_t gm = C >= 64 ? ~0ull : ((1ull << C) - 1);
  const bool surv = valid && q == 0 && ((rej >> (p << logC)) & gm) == 0;
  uint64_t sm = ballot(surv);
  if constexpr (CX::stats) cx.wide += (uint32_t)__builtin_popcountll(sm);
  while (sm) { // rare: no point proved below (a cell, a tie, or a point within the band)
    const int l = __builtin_ctzll(sm);
    sm &= sm - 1;
    decide_exact(cx, rl32(meta, l));
  }
#pragma unroll
  for (int i = 0; i < DENSE_TABLES; i++)
    cx.nd[i].recs -= (uint32_t)__builtin_popcountll(ballot(valid && q == 0 && t == cx.nd[i].t));
  cx.head = (cx.head + n) & (DENSE_RING - 1);
  cx.nrec -= n;
}

// 2^logC lanes per candidate for a last batch of n < 64 records
__device__ __forceinline__ int chunk_log(int n) {
  int logC = 0;
  while (logC < 6 && (n << (logC + 1)) <= 64) logC++;
  return logC;
}

// Lane mask of the bits [lo, hi) (lo <= hi <= 64).
__device__ __forceinline__ uint64_t bit_range(uint32_t lo, uint32_t hi) {
  const uint64_t below_hi = hi >= 64 ? ~0ull : (1ull << hi) - 1;
  const uint64_t below_lo = lo >= 64 ? ~0ull : (1ull << lo) - 1;
  return below_hi & ~below_lo;
}

// One setup pass: up to 64 pending triples, the oldest node's first, then
// the next ones'.  Each lane derives its triple's cofactors from its node's
// rows; the triples with D != 0 are appended to the record ring.
template <class CX>
__device__ __forceinline__ void setup_pass(CX &cx) {
  constexpr bool S = CX::stats;
  const int lane = lane_id();
  uint32_t cnt[DENSE_TABLES];
  uint32_t base = 0, r = 0;
  int t = cx.nd[0].t;
#pragma unroll
  for (int i = 0; i < DENSE_TABLES; i++) {
    NodeInfo &A = cx.nd[i];
    const uint32_t n = min(64u - base, A.r_hi - A.r_cur);
    if ((uint32_t)lane >= base && (uint32_t)lane < base + n) {
      t = A.t;
      r = A.r_cur + ((uint32_t)lane - base);
    }
    A.r_cur += n;
    cnt[i] = n;
    base += n;
  }
  const bool act = (uint32_t)lane < base;
  const TableInfo ti = cx.lds->info[t];
  Div dv;
  dv.e = ti.e;
  dv.inv = ti.inv;
  const bool prevneg = ti.prevneg != 0;
  int c1, c2, c3;
  unrank3(act ? r : 0, &c1, &c2, &c3); // (an inactive lane reads rows 2, 1, 0, in range)
  int64_t k0, k1, k2;
  int32_t D, d;
  triple_cofactors(cx.lds->rowS[t], cx.lds->rowH[t], c1, c2, c3, dv, prevneg, k0, k1, k2, D, d);
  const bool nz = act && D != 0;
  if constexpr (S) {
    cx.setups++;
    cx.triples += base;
  }
  const uint64_t m = ballot(nz);
  // the filter's shift: k_a >> sg within [-2^30, 2^30), and at least the table's
  const uint64_t mk = (uint64_t)(k0 ^ (k0 >> 63)) | (uint64_t)(k1 ^ (k1 >> 63)) | (uint64_t)(k2 ^ (k2 >> 63));
  const int sg = max(max(64 - __builtin_clzll(mk | 1) - 30, 0), (int)ti.sig);
  if (ballot(nz && sg > 0 && ti.band == BAND_UNSET)) {
    // a shifted record in a table whose band was not needed so far
    // (the band is taken eagerly for tables whose heights are shifted)
#pragma unroll
    for (int i = 0; i < DENSE_TABLES; i++)
      if (ballot(nz && sg > 0 && ti.band == BAND_UNSET && t == i)) {
        const int4 rw = cx.lds->rowS[i][lane];
        const uint32_t b = wave_umax((uint32_t)abs(rw.x) + (uint32_t)abs(rw.y) + (uint32_t)abs(rw.z));
        if (lane == 0) cx.lds->info[i].band = b;
      }
    wave_sync_lds();
  }
  if (nz) {
    const uint32_t below = (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1));
    const int slot = (cx.head + cx.nrec + (int)below) & (DENSE_RING - 1);
    cx.lds->recX[slot] = make_int4((int32_t)(k0 >> sg), (int32_t)(k1 >> sg), (int32_t)(k2 >> sg), d);
    cx.lds->recM[slot] = c1 | (c2 << 8) | (c3 << 16) | (t << REC_TABLE_BIT) | (sg << REC_SHIFT_BIT);
  }
  const int added = __builtin_popcountll(m);
  if constexpr (S) cx.leaves += (uint32_t)added;
  {
    uint32_t lo = 0;
#pragma unroll
    for (int i = 0; i < DENSE_TABLES; i++) {
      cx.nd[i].recs += (uint32_t)__builtin_popcountll(m & bit_range(lo, lo + cnt[i]));
      lo += cnt[i];
    }
  }
  cx.nrec += added;
  wave_sync_lds();
}

// Setup passes while at least `need` triples are pending (need = 1: all),
// each followed by a full test batch when 64 records wait.
template <class CX>
__device__ __forceinline__ bool run_setups(CX &cx, uint32_t need) {
  for (;;) {
    uint32_t pend = 0;
#pragma unroll
    for (int i = 0; i < DENSE_TABLES; i++) pend += cx.nd[i].r_hi - cx.nd[i].r_cur;
    if (pend == 0 || pend < need) return true;
    if (!charge(cx, 1)) return false;
    setup_pass(cx);
    if (cx.nrec >= 64) {
      if (!charge(cx, 1)) return false;
      test_batch(cx, 64, 0);
    }
  }
}

// Colex ranks [r_lo, r_hi) of the triples {c1 > c2 > c3} below `low` that
// complete the current node within the work unit's constraints (rank =
// C(c1,3) + C(c2,2) + c3; the unit fixes its top elements and restricts
// the element after them to [c_lo, c_hi]).
template <int K, class CX>
__device__ __forceinline__ void triple_range(const CX &cx, int low, uint32_t *rlo, uint32_t *rhi) {
  constexpr int P = K - 2; // position of c1 among the candidate's elements
  uint32_t r_lo = 0, r_hi = 0;
  {
    uint64_t below = cx.mask & ((1ull << low) - 1);
    if (cx.L < P) {
      r_hi = c3_of(low);
    } else if (cx.L == P) {
      const int lo = max(cx.c_lo, 2), hi = min(cx.c_hi, low - 1);
      if (hi >= lo) r_lo = c3_of(lo), r_hi = c3_of(hi + 1);
    } else {
      const int f1 = 63 - __builtin_clzll(below);
      below &= ~(1ull << f1);
      const uint32_t base1 = c3_of(f1);
      if (cx.L == P + 1) {
        const int lo = max(cx.c_lo, 1), hi = min(cx.c_hi, f1 - 1);
        if (hi >= lo) r_lo = base1 + c2_of(lo), r_hi = base1 + c2_of(hi + 1);
      } else {
        const int f2 = 63 - __builtin_clzll(below);
        below &= ~(1ull << f2);
        const uint32_t base2 = base1 + c2_of(f2);
        if (cx.L == P + 2) {
          const int lo = max(cx.c_lo, 0), hi = min(cx.c_hi, f2 - 1);
          if (hi >= lo) r_lo = base2 + (uint32_t)lo, r_hi = base2 + (uint32_t)hi + 1;
        } else {
          const int f3 = 63 - __builtin_clzll(below);
          r_lo = base2 + (uint32_t)f3, r_hi = r_lo + 1;
        }
      }
    }
  }
  *rlo = r_lo;
  *rhi = r_hi;
}

// A node with three spatial columns left (k - 2 points chosen, lowest
// `low`): its rows go into the table of the oldest node, after that node's
// triples and records are finished; its triples (within the work unit's
// constraints) join the pending ones, and full setup passes run.
template <int K, class CX>
__device__ __forceinline__ void triple_stage(CX &cx, const St<3> &st, int low) {
  const int lane = lane_id();
  const int t = cx.nd[0].t; // the oldest node's table is reused
  // 1. finish the oldest node
  {
    NodeInfo &O = cx.nd[0];
    while (O.r_cur < O.r_hi) {
      if (!charge(cx, 1)) return;
      setup_pass(cx);
      if (cx.nrec >= 64) {
        if (!charge(cx, 1)) return;
        test_batch(cx, 64, 0);
      }
    }
    if (O.recs > 0) { // at most 63 records wait, its own the oldest: test all
      if (!charge(cx, 1)) return;
      test_batch(cx, cx.nrec, chunk_log(cx.nrec));
    }
  }
  // 2. the node's rows (s0, s1, s2, h's low word, h split at bit 29)
  // (its heights' shift sig: the smallest with h >> sig in [-2^31, 2^31);
  // its band, the largest |s0| + |s1| + |s2|, now when sig > 0, else when a
  // record first needs it; padding lanes hold zeros)
  uint32_t sig = 0, band = BAND_UNSET;
  {
    const int64_t h = ((int64_t)st.H1 << 31) + (int64_t)st.H0;
    if (ballot(h != (int64_t)(int32_t)h) != 0) {
      sig = wave_umax((uint32_t)(64 - __builtin_clzll((uint64_t)(h ^ (h >> 63)) | 1))) - 31;
      band = wave_umax((uint32_t)abs(st.s[0]) + (uint32_t)abs(st.s[1]) + (uint32_t)abs(st.s[2]));
    }
    int4 r;
    r.x = st.s[0], r.y = st.s[1], r.z = st.s[2], r.w = (int32_t)(h >> sig);
    cx.lds->rowS[t][lane] = r;
    int2 hx;
    hx.x = (int32_t)(h >> DENSE_LIMB), hx.y = (int32_t)(h & DENSE_LMASK);
    cx.lds->rowH[t][lane] = hx;
  }
  if (lane == 0) {
    const Div dv = make_div(st.prev);
    TableInfo ti;
    ti.inv = dv.inv;
    ti.chosen = cx.chosen;
    ti.e = dv.e;
    ti.prevneg = st.prev < 0;
    ti.sig = sig;
    ti.band = band;
    cx.lds->info[t] = ti;
  }
  wave_sync_lds();
  // 3. colex ranks of the triples allowed below this node
  uint32_t r_lo, r_hi;
  triple_range<K>(cx, low, &r_lo, &r_hi);
  if constexpr (CX::stats) cx.nodes++;
#pragma unroll
  for (int i = 0; i + 1 < DENSE_TABLES; i++) cx.nd[i] = cx.nd[i + 1];
  {
    NodeInfo &Nn = cx.nd[DENSE_TABLES - 1];
    Nn.t = t;
    Nn.r_cur = r_lo;
    Nn.r_hi = r_hi > r_lo ? r_hi : r_lo;
    Nn.recs = 0;
  }
  // 4. full setup passes over the pending triples of the nodes in flight
  (void)run_setups(cx, 64);
}

// Cofactors of the tail quadruple {c0 > c1 > c2 > c3} from the rows in the
// tail table (all three levels divided exactly by the node's pivot): D, the
// spatial 4 x 4 minor, and kap_a = (-1)^a H_a, with row c3 taken times
// sign(D) sign(pivot) (so that a lower facet has every u_j > 0); d is D times
// the same sign.
__device__ __forceinline__ void quad_cofactors(const DenseLds *L, int c0, int c1, int c2, int c3, const Div &dv,
                                               bool prevneg, int64_t kap[4], int32_t &D, int32_t &d) {
  const int4 A = L->qS[c0], B = L->qS[c1], Cr = L->qS[c2], Dr = L->qS[c3];
  const int2 xa = L->qx[c0], xb = L->qx[c1], xc = L->qx[c2], xd = L->qx[c3];
  const int32_t a[4] = {A.x, A.y, A.z, A.w}, b[4] = {B.x, B.y, B.z, B.w};
  const int32_t c[4] = {Cr.x, Cr.y, Cr.z, Cr.w}, dd[4] = {Dr.x, Dr.y, Dr.z, Dr.w};
  // rows c0, c1: 2 x 2 minors (pairs 01 02 03 12 13 23) and with the height column
  int32_t m2[6];
  int64_t m2h[4];
  {
    int i = 0;
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int y = x + 1; y < 4; y++) m2[i++] = exdiv32((int64_t)a[x] * b[y] - (int64_t)a[y] * b[x], dv);
#pragma unroll
    for (int x = 0; x < 4; x++)
      m2h[x] = exdiv_limbs((int64_t)a[x] * xb.x - (int64_t)xa.x * b[x], (int64_t)a[x] * xb.y - (int64_t)xa.y * b[x], dv);
  }
  // pair index of {x < y}
  auto pi = [](int x, int y) { return x == 0 ? y - 1 : x == 1 ? y + 1 : 5; };
  // rows c0, c1, c2: 3 x 3 minors by expansion along row c2 (signs + - +):
  // spatial triples 012 013 023 123, and the pairs with the height column
  int32_t m3[4];
  int64_t m3h[6];
  {
    int i = 0;
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int y = x + 1; y < 4; y++)
#pragma unroll
        for (int z = y + 1; z < 4; z++)
          m3[i++] = exdiv32((int64_t)c[x] * m2[pi(y, z)] - (int64_t)c[y] * m2[pi(x, z)] + (int64_t)c[z] * m2[pi(x, y)], dv);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int y = x + 1; y < 4; y++) {
        int64_t Hi = (int64_t)xc.x * m2[pi(x, y)], Lo = (int64_t)xc.y * m2[pi(x, y)];
        acc_limbs(Hi, Lo, c[x], m2h[y]);
        acc_limbs(Hi, Lo, -c[y], m2h[x]);
        m3h[pi(x, y)] = exdiv_limbs(Hi, Lo, dv);
      }
  }
  // rows c0..c3: expansion along row c3 (signs - + - +); m3 index of the
  // spatial triple without column a: 3 - a
  D = exdiv32(-(int64_t)dd[0] * m3[3] + (int64_t)dd[1] * m3[2] - (int64_t)dd[2] * m3[1] + (int64_t)dd[3] * m3[0],
              dv);
  const bool flip = (D < 0) != prevneg;
  int32_t P[4];
#pragma unroll
  for (int x = 0; x < 4; x++) P[x] = flip ? -dd[x] : dd[x];
  const int32_t Ph = flip ? -xd.x : xd.x, Pl = flip ? -xd.y : xd.y;
  // kappa_a = (-1)^a H_a, H_a over the columns {0..3} \ {a} and h
#pragma unroll
  for (int del = 0; del < 4; del++) {
    int xs[3], m = 0;
#pragma unroll
    for (int x = 0; x < 4; x++)
      if (x != del) xs[m++] = x;
    const int32_t sgn = (del & 1) ? -1 : 1;
    int64_t Hi = (int64_t)(sgn * Ph) * m3[3 - del], Lo = (int64_t)(sgn * Pl) * m3[3 - del];
    acc_limbs(Hi, Lo, -sgn * P[xs[0]], m3h[pi(xs[1], xs[2])]);
    acc_limbs(Hi, Lo, sgn * P[xs[1]], m3h[pi(xs[0], xs[2])]);
    acc_limbs(Hi, Lo, -sgn * P[xs[2]], m3h[pi(xs[0], xs[1])]);
    kap[del] = exdiv_limbs(Hi, Lo, dv);
  }
  d = flip ? -D : D;
}

// The pivot of a tail child (its row r in the node's table): the first
// nonzero spatial column p (piv = 0 when there is none: a degenerate
// child), and the other three columns with their entries.
struct ChildPivot {
  int p;
  int32_t piv;
  int col[3];
  int32_t r[3];
};
__device__ __forceinline__ int32_t pick4(const int4 &v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
__device__ __forceinline__ ChildPivot child_pivot(const int4 R) {
  ChildPivot cp;
  cp.p = R.x != 0 ? 0 : R.y != 0 ? 1 : R.z != 0 ? 2 : 3;
  cp.piv = pick4(R, cp.p);
  cp.col[0] = cp.p == 0 ? 1 : 0;
  cp.col[1] = cp.p <= 1 ? 2 : 1;
  cp.col[2] = cp.p <= 2 ? 3 : 2;
#pragma unroll
  for (int i = 0; i < 3; i++) cp.r[i] = pick4(R, cp.col[i]);
  return cp;
}

// C(c, 4) for 3 <= c <= 7
__device__ __forceinline__ uint32_t c4_small(int c) { return c <= 3 ? 0u : c == 4 ? 1u : c == 5 ? 5u : c == 6 ? 15u : 35u; }

// The tail of a node with four spatial columns left (k - 3 points chosen):
// its children c in [lo_c, hi_c], all below DENSE_TAIL, would be nodes with
// at most C(6, 3) = 20 triples each.  Their candidates are instead the
// quadruples {c > c1 > c2 > c3} below DENSE_TAIL (at most C(7, 4) = 35),
// set up and tested in one pass from this node's rows, with no nodes of
// their own.  A quadruple's cofactors are the minors of its four rows
// (s0, s1, s2, s3, h) by three levels of Sylvester's identity, each
// divided exactly by the node's pivot:
//     u_j = H0 s0_j - H1 s1_j + H2 s2_j - H3 s3_j + D h_j = prev * M_j,
// H_a the 4 x 4 minor without column a, D the spatial one; the test is the
// filter of test_batch with five products, the survivors are decided
// exactly with lanes as points.
template <int K, class CX>
__device__ __forceinline__ void quad_tail(CX &cx, const St<4> &st, int lo_c, int hi_c) {
  constexpr bool S = CX::stats;
  const int lane = lane_id();
  // 1. colex ranks of the quadruples, rank = C(c,4) + C(c1,3) + C(c2,2) + c3
  uint32_t q_lo, q_hi;
  if (cx.L <= K - 3) { // c free (or within the unit's sibling run: [lo_c, hi_c] says so)
    q_lo = c4_small(lo_c);
    q_hi = c4_small(hi_c + 1);
  } else { // c fixed by the unit (lo_c == hi_c), the triple below it constrained
    uint32_t a, b;
    triple_range<K>(cx, lo_c, &a, &b);
    q_lo = c4_small(lo_c) + a;
    q_hi = c4_small(lo_c) + (b > a ? b : a);
  }
  if (q_hi <= q_lo) return;
  if (!charge(cx, 2)) return;
  const int n = (int)(q_hi - q_lo); // <= 35
  const int logC = chunk_log(n), C = 1 << logC;
  const int p = lane >> logC, q = lane & (C - 1);
  const bool act = p < n;
  // 2. the node's rows (its heights' shift sig and band as for a table)
  uint32_t sig = 0;
  {
    const int64_t h = ((int64_t)st.H1 << 31) + (int64_t)st.H0;
    if (ballot(h != (int64_t)(int32_t)h) != 0)
      sig = wave_umax((uint32_t)(64 - __builtin_clzll((uint64_t)(h ^ (h >> 63)) | 1))) - 31;
    cx.lds->qS[lane] = make_int4(st.s[0], st.s[1], st.s[2], st.s[3]);
    cx.lds->qh[lane] = (int32_t)(h >> sig);
    if (lane < DENSE_TAIL) cx.lds->qx[lane] = make_int2((int32_t)(h >> DENSE_LIMB), (int32_t)(h & DENSE_LMASK));
  }
  const uint32_t band = wave_umax((uint32_t)abs(st.s[0]) + (uint32_t)abs(st.s[1]) + (uint32_t)abs(st.s[2]) +
                                  (uint32_t)abs(st.s[3]));
  wave_sync_lds();
  const Div dv = make_div(st.prev);
  // 3. the children's rows, one Bareiss step each (lane C(c0,2) - 3 + x:
  //    child c0 < DENSE_TAIL, point x < c0), for the triple cofactors below
  {
    const int cc = 3 + (lane >= 3) + (lane >= 7) + (lane >= 12);
    const int x = lane - (int)(c2_of(cc) - 3u);
    if (lane < 18 && cc <= hi_c) {
      const ChildPivot cp = child_pivot(cx.lds->qS[cc]);
      const int4 Rx = cx.lds->qS[x];
      const int2 X0 = cx.lds->qx[cc], Xx = cx.lds->qx[x];
      const int32_t rxp = pick4(Rx, cp.p);
      int4 o;
      o.x = exdiv32((int64_t)cp.piv * pick4(Rx, cp.col[0]) - (int64_t)cp.r[0] * rxp, dv);
      o.y = exdiv32((int64_t)cp.piv * pick4(Rx, cp.col[1]) - (int64_t)cp.r[1] * rxp, dv);
      o.z = exdiv32((int64_t)cp.piv * pick4(Rx, cp.col[2]) - (int64_t)cp.r[2] * rxp, dv);
      o.w = 0;
      const int64_t hc = exdiv_limbs((int64_t)cp.piv * Xx.x - (int64_t)X0.x * rxp,
                                     (int64_t)cp.piv * Xx.y - (int64_t)X0.y * rxp, dv);
      cx.lds->ctS[lane] = o;
      cx.lds->ctH[lane] = make_int2((int32_t)(hc >> DENSE_LIMB), (int32_t)(hc & DENSE_LMASK));
    }
    wave_sync_lds();
  }
  // 4. lanes 2^logC p .. 2^logC p + 2^logC - 1 set up quadruple p (the same
  //    values in each; an inactive lane takes rank 0 = {3, 2, 1, 0}): the
  //    triple {c1, c2, c3} of child c0 (its pivot piv), whose coefficients
  //    k'_i over the child's columns turn into this node's: the same k'_i
  //    on the columns other than the child's pivot column p, and
  //    kap_p = -(sum_i k'_i R_c0[col_i] + d h_c0) / piv there (the child's
  //    residual of point j is (piv R_j - R_j[p] R_c0) / prev, so
  //    prev u'_j = piv u_j - R_j[p] (sum_i k'_i R_c0[col_i] + d h_c0), with
  //    u_j over this node's rows); the orientation then moves from
  //    sign(piv) to sign(prev).
  const uint32_t r = act ? q_lo + (uint32_t)p : 0u;
  const int c0 = 3 + (r >= 1) + (r >= 5) + (r >= 15);
  int c1, c2, c3;
  unrank3(r - c4_small(c0), &c1, &c2, &c3);
  int64_t kap[4];
  int32_t D, d;
  {
    const ChildPivot cp = child_pivot(cx.lds->qS[c0]);
    const Div dvc = make_div(cp.piv != 0 ? cp.piv : 1);
    const int b0 = (int)c2_of(c0) - 3;
    int64_t k[3];
    triple_cofactors(cx.lds->ctS, cx.lds->ctH, b0 + c1, b0 + c2, b0 + c3, dvc, cp.piv < 0, k[0], k[1], k[2], D, d);
    if (cp.piv == 0) D = 0; // the child is degenerate: every candidate below it has D = 0
    const int2 X0 = cx.lds->qx[c0];
    int64_t Hi = (int64_t)X0.x * d, Lo = (int64_t)X0.y * d;
    acc_limbs(Hi, Lo, cp.r[0], k[0]);
    acc_limbs(Hi, Lo, cp.r[1], k[1]);
    acc_limbs(Hi, Lo, cp.r[2], k[2]);
    const int64_t kp = -exdiv_limbs(Hi, Lo, dvc);
    const bool turn = (st.prev < 0) != (cp.piv < 0);
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int64_t v = c < cp.p ? (c < 3 ? k[c] : 0) : c == cp.p ? kp : k[c > 0 ? c - 1 : 0];
      kap[c] = turn ? -v : v;
    }
    d = turn ? -d : d;
  }
  const bool nz = act && D != 0;
  // 4. filter test (as in test_batch), 2^logC lanes per quadruple
  const uint64_t mk = (uint64_t)(kap[0] ^ (kap[0] >> 63)) | (uint64_t)(kap[1] ^ (kap[1] >> 63)) |
                      (uint64_t)(kap[2] ^ (kap[2] >> 63)) | (uint64_t)(kap[3] ^ (kap[3] >> 63));
  const int sg = max(max(64 - __builtin_clzll(mk | 1) - 30, 0), (int)sig);
  const int dl = sg - (int)sig;
  const int32_t x0 = (int32_t)(kap[0] >> sg), x1 = (int32_t)(kap[1] >> sg), x2 = (int32_t)(kap[2] >> sg),
                x3 = (int32_t)(kap[3] >> sg);
  const int64_t bnd = sg > 0 ? (int64_t)band + (d < 0 ? -(int64_t)d : (int64_t)d) - 1 : 0;
  const int iters = (cx.N + C - 1) >> logC;
  // Blocks of four points; the next block's rows are read before this
  // block's sums, so that the reads overlap the arithmetic.  Points past
  // the block count are zero rows or repeat row 63: harmless.
  int32_t neg = 0, first = 0;
  int4 cr[4];
  int32_t chh[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int j = min(q + (u << logC), 63);
    cr[u] = cx.lds->qS[j];
    chh[u] = cx.lds->qh[j];
  }
  for (int it0 = 0; it0 < iters; it0 += 4) {
    int4 nr[4];
    int32_t nh[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int j = min(q + ((it0 + 4 + u) << logC), 63);
      nr[u] = cx.lds->qS[j];
      nh[u] = cx.lds->qh[j];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int32_t hj = chh[u] >> dl;
      const int64_t v = bnd + (int64_t)cr[u].x * x0 + (int64_t)cr[u].y * x1 + (int64_t)cr[u].z * x2 +
                        (int64_t)cr[u].w * x3 + (int64_t)hj * d;
      neg |= (int32_t)((uint64_t)v >> 32);
      if constexpr (S)
        if (first == 0 && neg < 0) first = it0 + u + 1;
    }
    // one quadruple per lane: stop once each (with D != 0) has a point proved below
    if (logC == 0 && ballot(nz && neg >= 0) == 0) break;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      cr[u] = nr[u];
      chh[u] = nh[u];
    }
  }
  const uint64_t rej = ballot(neg < 0);
  const uint64_t gm = C >= 64 ? ~0ull : ((1ull << C) - 1);
  uint64_t sm = ballot(nz && q == 0 && ((rej >> (p << logC)) & gm) == 0);
  if constexpr (S) {
    cx.setups++;
    cx.tests++;
    cx.triples += (uint32_t)n;
    cx.quads += (uint32_t)n;
    cx.leaves += (uint32_t)__builtin_popcountll(ballot(nz && q == 0));
    cx.wide += (uint32_t)__builtin_popcountll(sm);
    if (nz && q == 0) cx.lpts += (uint32_t)((logC == 0 && first > 0) ? first : cx.N - cx.k - 1);
  }
  // 5. survivors: exact, lanes as points with this node's rows in registers
  if (sm) {
    const int64_t h = ((int64_t)st.H1 << 31) + (int64_t)st.H0;
    const int32_t hh = (int32_t)(h >> DENSE_LIMB), hl = (int32_t)(h & DENSE_LMASK);
    const uint32_t vpack = (uint32_t)c0 | ((uint32_t)c1 << 8) | ((uint32_t)c2 << 16) | ((uint32_t)c3 << 24);
    while (sm) {
      const int l = __builtin_ctzll(sm);
      sm &= sm - 1;
      // (the exact cofactors again, for this one quadruple: rarely needed,
      // so not kept in registers through the test)
      const uint32_t vp = (uint32_t)rl32((int32_t)vpack, l);
      int64_t kx[4];
      int32_t Dx, dl_;
      quad_cofactors(cx.lds, (int)(vp & 255), (int)((vp >> 8) & 255), (int)((vp >> 16) & 255), (int)(vp >> 24), dv,
                     st.prev < 0, kx, Dx, dl_);
      int32_t kl[4], kh[4];
#pragma unroll
      for (int x = 0; x < 4; x++) {
        kl[x] = (int32_t)(kx[x] & DENSE_LMASK);
        kh[x] = (int32_t)(kx[x] >> DENSE_LIMB);
      }
      const int64_t lo = (int64_t)st.s[0] * kl[0] + (int64_t)st.s[1] * kl[1] + (int64_t)st.s[2] * kl[2] +
                         (int64_t)st.s[3] * kl[3] + (int64_t)hl * dl_;
      const int64_t hi = (lo >> DENSE_LIMB) + (int64_t)st.s[0] * kh[0] + (int64_t)st.s[1] * kh[1] +
                         (int64_t)st.s[2] * kh[2] + (int64_t)st.s[3] * kh[3] + (int64_t)hh * dl_;
      const bool in = cx.j < cx.N;
      if (ballot(in && hi < 0)) continue; // a point below within the filter's band
      const uint64_t zero = ballot(in && hi == 0 && (lo & DENSE_LMASK) == 0);
      const uint64_t verts = cx.chosen | (1ull << (vp & 255)) | (1ull << ((vp >> 8) & 255)) |
                             (1ull << ((vp >> 16) & 255)) | (1ull << (vp >> 24));
      if (zero != verts) {
        if (lane == 0) cx.lds->tally.tie = 1;
        continue;
      }
      if (lane == 0) {
        cx.lds->tally.acc += (unsigned long long)(dl_ < 0 ? -(int64_t)dl_ : (int64_t)dl_);
        cx.lds->tally.cells += 1;
      }
      if constexpr (CX::emit) emit_cell(cx, unlabel(cx, verts));
    }
  }
}

// End of a work unit: every pending triple and record.
template <class CX>
__device__ __forceinline__ void dense_flush(CX &cx) {
  if (!run_setups(cx, 1)) return;
  while (cx.nrec > 0) {
    if (!charge(cx, 1)) return;
    const int n = cx.nrec < 64 ? cx.nrec : 64;
    test_batch(cx, n, n < 64 ? chunk_log(n) : 0);
  }
}

// Range of the next element at depth T (as next_range in enum_device.hpp).
template <class CX>
__device__ __forceinline__ void dense_next_range(const CX &cx, int T, int K, int low, int *hi_c, int *lo_c) {
  if (T + 1 < cx.L) {
    const uint64_t below = cx.mask & ((1ull << low) - 1);
    *hi_c = *lo_c = 63 - __builtin_clzll(below);
    return;
  }
  *hi_c = low - 1;
  *lo_c = K - T - 1;
  if (T + 1 == cx.L) {
    *hi_c = min(*hi_c, cx.c_hi);
    *lo_c = max(*lo_c, cx.c_lo);
  }
}

// st holds depth T (T+1 points chosen, lowest `low`), W = K - T >= 3 columns.
template <int K, int T, class CX>
struct DLevel {
  static __device__ __forceinline__ void run(CX &cx, const St<K - T> &st, int low) {
    constexpr int W = K - T;
    if constexpr (W == 3) {
      triple_stage<K>(cx, st, low);
    } else {
      int hi_c, lo_c;
      dense_next_range(cx, T, K, low, &hi_c, &lo_c);
      // with four columns left, the children below DENSE_TAIL are the tail
      const int c_end = W == 4 ? max(lo_c, DENSE_TAIL) : lo_c;
      for (int c = hi_c; c >= c_end && step_ok(cx); --c) {
        int32_t rc[W];
#pragma unroll
        for (int i = 0; i < W; i++) rc[i] = rl32(st.s[i], c);
        int p = -1;
#pragma unroll
        for (int i = 0; i < W; i++)
          if (p < 0 && rc[i] != 0) p = i;
        if (p < 0) { // affinely dependent on the prefix: D = 0 below
          if constexpr (CX::stats) cx.pruned++;
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
        const Div dv = make_div(st.prev);
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
        if constexpr (CX::stats) {
          cx.inner++;
          cx.sp_upd += W - 1;
        }
        cx.chosen |= 1ull << c;
        DLevel<K, T + 1, CX>::run(cx, ch, c);
        cx.chosen &= ~(1ull << c);
      }
      if constexpr (W == 4)
        if (lo_c < DENSE_TAIL && hi_c >= lo_c) quad_tail<K>(cx, st, lo_c, min(hi_c, DENSE_TAIL - 1));
    }
  }
};

template <int K, class CX>
__device__ __forceinline__ void dense_tile(CX &cx, const SysDesc &sd, const int32_t *__restrict__ pts,
                                           const int64_t *__restrict__ hts) {
  const bool valid = cx.j < sd.N;
  int32_t P[K];
  int64_t w = 0;
#pragma unroll
  for (int i = 0; i < K; i++) P[i] = 0;
  if (valid) {
    const int src = cx.lds->perm[cx.j];
#pragma unroll
    for (int i = 0; i < K; i++) P[i] = pts[sd.pt_off + src * K + i];
    w = hts[sd.ht_off + src];
  }
  const int base = 63 - __builtin_clzll(cx.mask);
  const int64_t wb = (int64_t)(((uint64_t)(uint32_t)rl32((int32_t)(uint32_t)((uint64_t)w >> 32), base) << 32) |
                               (uint32_t)rl32((int32_t)(uint32_t)w, base));
  const int64_t h0 = valid ? w - wb : 0; // padding lanes: zero rows
  St<K> st;
#pragma unroll
  for (int i = 0; i < K; i++) st.s[i] = valid ? P[i] - rl32(P[i], base) : 0;
  st.H1 = (int32_t)(h0 >> 31);
  st.H0 = (int32_t)((uint32_t)h0 & LOW31);
  st.prev = 1;
  cx.chosen = 1ull << base;
  DLevel<K, 0, CX>::run(cx, st, base);
}

// Add the wave's tally (the unit's lower facets, plus those of earlier
// units' candidates decided during it) and work counts to the system's
// accumulators, and clear them; a unit that ran out of steps reports an error.
template <class CX>
__device__ __forceinline__ void dense_commit(CX &cx, const SysDesc &sd, SysAcc *a, DevCounters *cnt, bool unit) {
  constexpr bool S = CX::stats;
  const int lane = lane_id();
  uint32_t lpts = 0;
  if constexpr (S) lpts = wave_usum(cx.lpts);
  wave_sync_lds();
  const bool abandoned = cx.left <= 0;
  if (lane == 0 && abandoned) atomicOr(&cnt->error, 1u);
  if (lane == 0 && !abandoned) {
    const unsigned long long sum = cx.lds->tally.acc;
    const uint32_t cells = cx.lds->tally.cells, tie = cx.lds->tally.tie;
    if (sum | cells | tie) {
      const unsigned long long old = atomicAdd((unsigned long long *)&a->lo, sum);
      if (old + sum < old) atomicAdd((unsigned long long *)&a->hi, 1ull);
      atomicAdd((unsigned long long *)&a->cells, (unsigned long long)cells);
      if (tie) atomicOr(&a->tie, 1u);
    }
    if constexpr (S) {
      const unsigned long long n = (unsigned long long)sd.N;
      atomicAdd((unsigned long long *)&cnt->inner, (unsigned long long)cx.inner);
      atomicAdd((unsigned long long *)&cnt->sp_upd, (unsigned long long)cx.sp_upd);
      atomicAdd((unsigned long long *)&cnt->pruned, (unsigned long long)cx.pruned);
      // (no ridges in this schedule: its nodes with three spatial columns
      // left, setup passes, test batches and the candidates decided exactly
      // after the batch test take the ridge, ridge-step, leaf-step and
      // empty-step counters)
      atomicAdd((unsigned long long *)&cnt->leaves, (unsigned long long)cx.leaves);
      atomicAdd((unsigned long long *)&cnt->rsteps, (unsigned long long)cx.setups);
      atomicAdd((unsigned long long *)&cnt->lsteps, (unsigned long long)cx.tests);
      atomicAdd((unsigned long long *)&cnt->triples, (unsigned long long)cx.triples);
      atomicAdd((unsigned long long *)&cnt->quads, (unsigned long long)cx.quads);
      atomicAdd((unsigned long long *)&cnt->lempty, (unsigned long long)cx.wide);
      atomicAdd((unsigned long long *)&cnt->ridges, (unsigned long long)cx.nodes);
      if (unit) {
        atomicAdd((unsigned long long *)&cnt->dunits, 1ull);
        atomicAdd((unsigned long long *)&cnt->tiles, 1ull);
      }
      atomicAdd((unsigned long long *)&cnt->w_inner, n * cx.inner);
      atomicAdd((unsigned long long *)&cnt->w_spatial, n * cx.sp_upd);
      atomicAdd((unsigned long long *)&cnt->w_leaves, (unsigned long long)lpts);
    }
    cx.lds->tally.acc = 0;
    cx.lds->tally.cells = 0;
    cx.lds->tally.tie = 0;
  }
  cx.inner = cx.sp_upd = cx.pruned = cx.nodes = cx.triples = cx.leaves = cx.setups = cx.tests = cx.wide = cx.quads = cx.lpts = 0;
  wave_sync_lds();
}

// The depth-first walk of one work unit.  The setup and test pipeline is
// not drained at its end: the next unit of the same system goes on with the
// pending triples and records (their rows stay in the tables), so that the
// passes and batches stay full across unit boundaries.
template <int KLO, int KHI, class CX>
__device__ __forceinline__ void dense_unit(CX &cx, const Tile &tl, const SysDesc &sd, const int32_t *__restrict__ pts,
                                           const int64_t *__restrict__ hts) {
  cx.mask = tl.mask;
  cx.L = __builtin_popcountll(tl.mask);
  cx.c_lo = tl.c_lo;
  cx.c_hi = tl.c_hi;
  {
    // (k + 3) steps per candidate, plus room for the passes and batches of
    // up to 64 + 64 candidates carried over from the previous unit
    const uint64_t cand = unit_candidates(sd.k, tl.mask, tl.c_lo, tl.c_hi);
    const uint64_t b = cand * (uint64_t)(sd.k + 3) + 256;
    cx.left = b > 0x7FFFFFF0ull ? 0x7FFFFFF0 : (int32_t)b;
  }
  switch (sd.k) {
#define BDEG_DCASE(KK)                                     \
  case KK:                                                 \
    if constexpr (KK >= KLO && KK <= KHI && KK >= 3)       \
      dense_tile<KK, CX>(cx, sd, pts, hts);                \
    break;
    BDEG_DCASE(3) BDEG_DCASE(4) BDEG_DCASE(5) BDEG_DCASE(6) BDEG_DCASE(7) BDEG_DCASE(8)
    BDEG_DCASE(9) BDEG_DCASE(10) BDEG_DCASE(11) BDEG_DCASE(12) BDEG_DCASE(13) BDEG_DCASE(14)
    BDEG_DCASE(15) BDEG_DCASE(16) BDEG_DCASE(17) BDEG_DCASE(18)
#undef BDEG_DCASE
    default:
      break;
  }
}

// Waves per SIMD the dense kernel is compiled for: the depth-first states
// above the triple stage grow with k (about (k^2 + 7k) / 2 registers), the
// triple stage adds a fixed working set; four waves is also the LDS limit
// (34.4 KiB per block of four waves, four blocks per compute unit).
constexpr int dense_waves(int k) { return k <= 10 ? 4 : k <= 13 ? 3 : 2; }

template <int KLO, int KHI, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dense_waves(KHI))))
dense_kernel(const SysDesc *__restrict__ sys, const int32_t *__restrict__ pts, const int64_t *__restrict__ hts,
             const Tile *__restrict__ tiles, uint32_t n_tiles, SysAcc *__restrict__ acc,
             DevCounters *__restrict__ cnt, CellSink sink, const uint32_t *__restrict__ rerun) {
  const int lane = lane_id();
  __shared__ DenseLds lds_all[4]; // one per wavefront of the block (at most 256 threads)
  DenseLds *lds = &lds_all[threadIdx.x >> 6];
  if (rerun && rerun[0] == 0) return;
  using CX = DCtx<MODE>;
  CX cx;
  cx.j = lane;
  cx.lds = lds;
  cx.sink = sink;
  cx.head = 0;
  cx.nrec = 0;
#pragma unroll
  for (int i = 0; i < DENSE_TABLES; i++) {
    cx.nd[i].t = i;
    cx.nd[i].r_cur = cx.nd[i].r_hi = 0;
    cx.nd[i].recs = 0;
  }
  cx.inner = cx.sp_upd = cx.pruned = cx.nodes = cx.triples = cx.leaves = cx.setups = cx.tests = cx.wide = cx.quads = cx.lpts = 0;
  cx.left = 1;
  if (lane == 0) {
    lds->tally.acc = 0;
    lds->tally.cells = 0;
    lds->tally.tie = 0;
  }
  uint32_t cur_sys = 0xFFFFFFFFu;
  SysDesc sd{};
  for (;;) {
    // every lane joins the claim; lane 0's result is read by index (no
    // lane-dependent branch around the loop's exit test)
    const uint32_t claim = atomicAdd(&cnt->next_tile, lane == 0 ? 1u : 0u);
    const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int32_t)claim, 0);
    if (t >= n_tiles) break;
    const Tile tl = tiles[t];
    if (rerun && rerun[1 + tl.sys] == 0) continue;
    if (tl.sys != cur_sys) {
      if (cur_sys != 0xFFFFFFFFu) { // another system: finish the previous one's candidates
        cx.left = 256;
        dense_flush(cx);
        dense_commit(cx, sd, &acc[cur_sys], cnt, false);
      }
      cur_sys = tl.sys;
      sd = sys[tl.sys];
      cx.N = sd.N;
      cx.k = sd.k;
      dense_order(cx, sd, hts);
    }
    dense_unit<KLO, KHI>(cx, tl, sd, pts, hts);
    dense_commit(cx, sd, &acc[cur_sys], cnt, true);
  }
  if (cur_sys != 0xFFFFFFFFu) {
    cx.left = 256;
    dense_flush(cx);
    dense_commit(cx, sd, &acc[cur_sys], cnt, false);
  }
}

} // namespace dev
} // namespace bdeg

// Instantiation helper: one translation unit per k range defines
// bdeg::enum_fn_<klo>_<khi>(mode, variant) for the three kernel variants
// (0: lane groups read per system, 1: one point group per wavefront, 2: the
// lane-dense kernel, k >= 3).  The emitting mode exists for single-k kernels
// only.
namespace bdeg {
namespace dev {
template <int KLO, int KHI>
EnumFn pick_dense(int mode) {
  if constexpr (KHI < 3) {
    return nullptr;
  } else {
    if (mode == MODE_STATS) return dense_kernel<KLO, KHI, MODE_STATS>;
    if (mode == MODE_EMIT) {
      if constexpr (KLO == KHI) return dense_kernel<KLO, KHI, MODE_EMIT>;
      else return nullptr;
    }
    return dense_kernel<KLO, KHI, MODE_PLAIN>;
  }
}
} // namespace dev
} // namespace bdeg

#define BDEG_ENUM_INSTANCES(KLO, KHI)                                                         \
  namespace bdeg {                                                                            \
  EnumFn enum_fn_##KLO##_##KHI(int mode, int variant) {                                       \
    return variant == 2 ? dev::pick_dense<KLO, KHI>(mode) : dev::pick_kernel<KLO, KHI>(mode, variant == 1); \
  }                                                                                           \
  }
