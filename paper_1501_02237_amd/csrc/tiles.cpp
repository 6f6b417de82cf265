// Work decomposition of the candidate space of one system.
//
// Candidates are the (k+1)-subsets {c_0 < ... < c_k} of the N points (the
// brute-force search over all subsets of Section 4), numbered in colex order
// rank = sum_i C(c_i, i+1).  Fixing the top elements c_k > ... > c_{k-L+1}
// (a "prefix" of L elements, lowest element e) leaves C(e, k+1-L) completions
// whose ranks form one contiguous interval; such a subtree is one device work
// unit, described by the bit mask of its prefix.
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "bdeg_internal.hpp"

namespace bdeg {

// C(n, r) for 0 <= n, r <= 64, saturated at UINT64_MAX (computed once).
namespace {
struct BinomTable {
  uint64_t c[65][65];
  BinomTable() {
    for (int n = 0; n <= 64; n++)
      for (int r = 0; r <= 64; r++) {
        if (r > n) {
          c[n][r] = 0;
        } else if (r == 0 || r == n) {
          c[n][r] = 1;
        } else {
          const uint64_t a = c[n - 1][r - 1], b = c[n - 1][r];
          c[n][r] = (a > UINT64_MAX - b) ? UINT64_MAX : a + b;
        }
      }
  }
};
const BinomTable &binom_table() {
  static const BinomTable t;
  return t;
}
} // namespace

uint64_t binom_u64(int n, int r) {
  if (r < 0 || n < 0 || r > n) return 0;
  if (n <= 64) return binom_table().c[n][r];
  if (r > n - r) r = n - r;
  u128 c = 1;
  for (int i = 1; i <= r; i++) {
    c = c * (u128)(n - r + i) / (u128)i;
    if (c > (u128)UINT64_MAX) return UINT64_MAX;
  }
  return (uint64_t)c;
}

static void emit(std::vector<TileC> &out, uint32_t sys, uint64_t mask, int c_lo, int c_hi, uint64_t cost) {
  TileC t;
  t.t.mask = mask;
  t.t.sys = sys;
  t.t.c_lo = (uint8_t)c_lo;
  t.t.c_hi = (uint8_t)c_hi;
  t.t.pad = 0;
  t.cost = cost;
  out.push_back(t);
}

// prefix `mask` has L elements with lowest element e; its subtree has
// C(e, k+1-L) candidates.  A subtree above max_cost is split into its
// children (next element c, C(c, k-L) candidates each); children at or below
// max_cost are grouped into runs of consecutive siblings of total cost at
// most max_cost, so that one work unit derives the shared prefix once.
// A k-point prefix (a ridge, at most e <= 63 leaves) is never split.
static void split(int k, uint32_t sys, uint64_t mask, int L, int e, uint64_t max_cost, std::vector<TileC> &out) {
  uint64_t cost = binom_u64(e, k + 1 - L);
  if (cost == 0) return;
  if (cost <= max_cost || L >= k) {
    emit(out, sys, mask, 0, 63, cost);
    return;
  }
  int run_hi = -1, run_lo = -1;
  uint64_t run_cost = 0;
  auto flush = [&]() {
    if (run_hi >= 0) emit(out, sys, mask, run_lo, run_hi, run_cost);
    run_hi = run_lo = -1;
    run_cost = 0;
  };
  for (int c = e - 1; c >= k - L; c--) {
    uint64_t cc = binom_u64(c, k - L);
    if (cc == 0) continue;
    if (cc > max_cost) {
      flush();
      split(k, sys, mask | (1ull << c), L + 1, c, max_cost, out);
      continue;
    }
    if (run_hi >= 0 && run_cost + cc > max_cost) flush();
    if (run_hi < 0) run_hi = c;
    run_lo = c;
    run_cost += cc;
  }
  flush();
}

void tiles_full(int N, int k, uint32_t sys, uint64_t max_cost, std::vector<TileC> &out) {
  if (max_cost == 0) max_cost = 1;
  // every work unit fixes at least the top element b (a kernel needs a base
  // point), so the top elements are never grouped
  for (int b = N - 1; b >= k; b--) split(k, sys, 1ull << b, 1, b, max_cost, out);
}

// Ranks of the children of a node: the next element c (position i = k - L)
// covers [base + C(c, i+1), base + C(c+1, i+1)).
static void cover(int k, uint32_t sys, uint64_t mask, int L, int e, uint64_t base, uint64_t lo, uint64_t hi,
                  uint64_t max_cost, std::vector<TileC> &out) {
  const int i = k - L;
  for (int c = i; c < e; c++) {
    uint64_t start = base + binom_u64(c, i + 1);
    uint64_t size = binom_u64(c, i);
    uint64_t end = start + size;
    if (end <= lo || start >= hi) continue;
    uint64_t m2 = mask | (1ull << c);
    if (lo <= start && end <= hi)
      split(k, sys, m2, L + 1, c, max_cost, out);
    else
      cover(k, sys, m2, L + 1, c, start, lo, hi, max_cost, out);
  }
}

void tiles_range(int N, int k, uint32_t sys, uint64_t lo, uint64_t hi, uint64_t max_cost, std::vector<TileC> &out) {
  uint64_t total = binom_u64(N, k + 1);
  if (hi > total) hi = total;
  if (lo >= hi) return;
  if (max_cost == 0) max_cost = 1;
  cover(k, sys, 0, 0, N, 0, lo, hi, max_cost, out);
}

// colex rank interval of a work unit
void tile_interval(const Tile &t, int k, uint64_t *start, uint64_t *end) {
  uint64_t base = 0, m = t.mask;
  int L = 0, e = 64;
  while (m) {
    const int c = 63 - __builtin_clzll(m);
    base += binom_u64(c, k + 1 - L); // element at colex position k - L
    m &= ~(1ull << c);
    e = c;
    L++;
  }
  const int i = k - L; // position of the next element
  if (L == k + 1) {
    *start = base;
    *end = base + 1;
    return;
  }
  int hi = std::min(e - 1, (int)t.c_hi), lo = std::max(i, (int)t.c_lo);
  *start = base + binom_u64(lo, i + 1);
  *end = base + binom_u64(hi + 1, i + 1);
}

void tiles_sorted(std::vector<TileC> &in, std::vector<Tile> &out) {
  std::stable_sort(in.begin(), in.end(), [](const TileC &a, const TileC &b) { return a.cost > b.cost; });
  out.resize(in.size());
  for (size_t i = 0; i < in.size(); i++) out[i] = in[i].t;
}

} // namespace bdeg
