// Host side of the cell walk (simplicial pivoting, paper Section 4.2-4.4):
// device buffers, the level-by-level launch loop and the C-ABI entry points.
//
// The walk starts from a cell that is a lower facet for the given heights and
// visits the cells breadth-first: every level is one persistent launch over
// the cells discovered by the previous level; the host reads the work-list
// length between levels (no device-side waiting).  A wavefront also follows
// a chain of new neighbours by single pivots; those cells skip the list.  A
// tie is returned to the caller.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "api_internal.hpp"
#include "runtime.hpp"

namespace bdeg {
namespace {

uint64_t host_cell_hash(uint64_t m) { // same mixing as the device hash set
  m ^= m >> 33;
  m *= 0xFF51AFD7ED558CCDull;
  m ^= m >> 33;
  m *= 0xC4CEB9FE1A85EC53ull;
  m ^= m >> 33;
  return m;
}

struct WalkBuffers {
  int32_t *pts = nullptr;
  int64_t *hts = nullptr;
  uint64_t *list = nullptr, *table = nullptr;
  PivotCounters *cnt = nullptr;
  uint64_t cap = 0; // cells (work list and hash set; the set has 2 * cap slots)
  void release() {
    for (void *p : {(void *)pts, (void *)hts, (void *)list, (void *)table, (void *)cnt})
      if (p) (void)hipFree(p);
    pts = nullptr;
    hts = nullptr;
    list = table = nullptr;
    cnt = nullptr;
    cap = 0;
  }
  ~WalkBuffers() { release(); }
};

struct WalkResult {
  u128 nvol = 0;
  uint64_t cells = 0;
  bool tie = false;
  uint64_t start = 0; // the start cell (the caller's, or the one Extend found)
};

// Cells of the walk with their inner normals (alpha, 1), alpha = num / den.
struct CellNormals {
  std::vector<uint64_t> masks;
  std::vector<int64_t> num; // k per cell
  std::vector<uint64_t> den;
};

// Extend on the device: a lower facet of the uploaded points and heights.
int extend_device(Device *D, const int32_t *d_pts, const int64_t *d_hts, int N, int k, uint64_t *mask, bool *tie) {
  ExtendResult *d_out = nullptr;
  if (hipMalloc((void **)&d_out, sizeof(ExtendResult)) != hipSuccess) return BDEG_E_NOMEM;
  ExtendResult r{};
  int rc = launch_extend(D->stream, d_pts, d_hts, N, k, d_out);
  if (!rc && (hipMemcpyAsync(&r, d_out, sizeof r, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
              hipStreamSynchronize(D->stream) != hipSuccess))
    rc = BDEG_E_DEVICE;
  (void)hipFree(d_out);
  if (rc) return rc;
  if (r.flags & EXTEND_ERR_RANGE) return BDEG_E_OVERFLOW;
  if (r.flags & EXTEND_ERR_SPAN) return BDEG_E_ARG;
  *tie = (r.flags & EXTEND_TIE) != 0;
  *mask = r.mask;
  if (!*tie && __builtin_popcountll(r.mask) != k + 1) return BDEG_E_STATE;
  return BDEG_OK;
}

// Inner normals of listed cells (the cell-list kernel of the enumeration path).
int normals_device(Device *D, const int32_t *d_pts, const int64_t *d_hts, int N, int k, CellNormals &c) {
  const uint64_t n = c.masks.size();
  c.num.assign(n * k, 0);
  c.den.assign(n, 0);
  if (n == 0) return BDEG_OK;
  uint64_t *d_masks = nullptr, *d_den = nullptr;
  int64_t *d_num = nullptr;
  uint32_t *d_err = nullptr;
  int rc = BDEG_OK;
  if (hipMalloc((void **)&d_masks, n * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc((void **)&d_den, n * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc((void **)&d_num, n * (size_t)k * sizeof(int64_t)) != hipSuccess ||
      hipMalloc((void **)&d_err, sizeof(uint32_t)) != hipSuccess)
    rc = BDEG_E_NOMEM;
  uint32_t err = 0;
  if (!rc && (hipMemcpyAsync(d_masks, c.masks.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice, D->stream) !=
                  hipSuccess ||
              hipMemcpyAsync(d_err, &err, sizeof err, hipMemcpyHostToDevice, D->stream) != hipSuccess))
    rc = BDEG_E_DEVICE;
  if (!rc) rc = launch_cell_normals(D->stream, d_masks, n, d_pts, d_hts, N, k, d_num, d_den, d_err);
  if (!rc && (hipMemcpyAsync(c.num.data(), d_num, n * (size_t)k * sizeof(int64_t), hipMemcpyDeviceToHost,
                             D->stream) != hipSuccess ||
              hipMemcpyAsync(c.den.data(), d_den, n * sizeof(uint64_t), hipMemcpyDeviceToHost, D->stream) !=
                  hipSuccess ||
              hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
              hipStreamSynchronize(D->stream) != hipSuccess))
    rc = BDEG_E_DEVICE;
  for (void *p : {(void *)d_masks, (void *)d_den, (void *)d_num, (void *)d_err})
    if (p) (void)hipFree(p);
  if (!rc && (err & 1u)) rc = BDEG_E_DEVICE;   // a listed mask is not a (k+1)-subset
  if (!rc && (err & 2u)) rc = BDEG_E_OVERFLOW; // a value outside the certified widths
  return rc;
}

// Make room for `need` cells: a larger work list (the listed cells copied)
// and a hash set of twice that many slots rebuilt from the old set (it holds
// every cell, also those reached by pivots that never enter the list), so the set's
// load stays at most 1/2.
int grow(Device *D, WalkBuffers &b, PivotArgs &a, uint64_t need, uint32_t tail) {
  uint64_t cap = b.cap ? b.cap : (1ull << 20);
  while (cap < need) cap *= 2;
  if (cap > (1ull << 31)) return BDEG_E_NOMEM; // work-list indices are 32-bit
  if (cap == b.cap) return BDEG_OK;
  uint64_t *list = nullptr, *table = nullptr;
  if (hipMalloc((void **)&list, cap * sizeof(uint64_t)) != hipSuccess) return BDEG_E_NOMEM;
  if (hipMalloc((void **)&table, 2 * cap * sizeof(uint64_t)) != hipSuccess) {
    (void)hipFree(list);
    return BDEG_E_NOMEM;
  }
  a.list = list;
  a.cap_list = (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFFFull);
  a.table = table;
  a.table_mask = 2 * cap - 1;
  int rc = BDEG_OK;
  if (hipMemsetAsync(table, 0, 2 * cap * sizeof(uint64_t), D->stream) != hipSuccess ||
      (tail && hipMemcpyAsync(list, b.list, tail * sizeof(uint64_t), hipMemcpyDeviceToDevice, D->stream) !=
                   hipSuccess))
    rc = BDEG_E_DEVICE;
  if (!rc && b.table) rc = launch_pivot_rehash(D->stream, a, b.table, 2 * b.cap);
  if (!rc && hipStreamSynchronize(D->stream) != hipSuccess) rc = BDEG_E_DEVICE;
  if (rc) {
    (void)hipFree(list);
    (void)hipFree(table);
    return rc;
  }
  if (b.list) (void)hipFree(b.list);
  if (b.table) (void)hipFree(b.table);
  b.list = list;
  b.table = table;
  b.cap = cap;
  return BDEG_OK;
}

// One walk from `start`, breadth first.  Before each level the list and the
// set are grown to the level's worst case (every processed cell adds at most
// k + 1 new ones), so a level never runs out of room; a probe sequence that
// runs out anyway (PIVOT_ERR_FULL) restarts the walk with twice the room.
// start == 0: the start cell is found by Extend; a tie there is returned as
// a tie of the walk.  With `normals`, the cells and their inner normals are
// returned too.
int walk(Device *D, const int32_t *points, const int64_t *heights, int N, int k, uint64_t start,
         std::vector<uint64_t> *cells_out, WalkResult &out, CellNormals *normals = nullptr) {
  WalkBuffers b;
  if (hipMalloc((void **)&b.pts, (size_t)N * k * sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void **)&b.hts, (size_t)N * sizeof(int64_t)) != hipSuccess ||
      hipMalloc((void **)&b.cnt, sizeof(PivotCounters)) != hipSuccess)
    return BDEG_E_NOMEM;
  if (hipMemcpy(b.pts, points, (size_t)N * k * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b.hts, heights, (size_t)N * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
    return BDEG_E_DEVICE;
  const int blocks = max_pivot_blocks(k);
  if (blocks <= 0) return BDEG_E_DEVICE;
  if (start == 0) {
    bool tie = false;
    const int rc = extend_device(D, b.pts, b.hts, N, k, &start, &tie);
    if (rc) return rc;
    if (tie) {
      out.tie = true;
      return BDEG_OK;
    }
  }
  out.start = start;
  std::vector<uint64_t> own;
  if (normals && !cells_out) cells_out = &own;
  for (uint64_t room = 1ull << 20;; room *= 2) {
    if (room > (1ull << 31)) return BDEG_E_NOMEM;
    PivotArgs a;
    a.pts = b.pts;
    a.hts = b.hts;
    a.N = N;
    a.cnt = b.cnt;
    // a fresh, empty list and set of `room` cells holding the start cell
    if (b.list) (void)hipFree(b.list);
    if (b.table) (void)hipFree(b.table);
    b.list = b.table = nullptr;
    b.cap = 0;
    int rc = grow(D, b, a, room, 0);
    if (rc) return rc;
    PivotCounters c0{};
    c0.tail = 1;
    if (hipMemcpyAsync(b.list, &start, sizeof start, hipMemcpyHostToDevice, D->stream) != hipSuccess ||
        hipMemcpyAsync(b.table + (host_cell_hash(start) & a.table_mask), &start, sizeof start,
                       hipMemcpyHostToDevice, D->stream) != hipSuccess ||
        hipMemcpyAsync(b.cnt, &c0, sizeof c0, hipMemcpyHostToDevice, D->stream) != hipSuccess)
      return BDEG_E_DEVICE;
    uint32_t first = 0, count = 1;
    uint64_t in_set = 1; // cells in the set: the listed ones and those reached by pivots
    PivotCounters c{};
    bool regrow = false;
    while (count > 0) {
      // every cell processed in this level (listed, or reached by a pivot)
      // inserts at most k + 1 new cells into the set and the list; room for
      // the listed cells' worst case (twice over while that fits in 2^31
      // cells, else a quarter more), and pivots reserved only within the
      // room left, keep the list within its capacity and the set at most
      // half full
      const uint64_t tail0 = (uint64_t)first + count;
      const uint64_t worst = (uint64_t)count * (k + 1);
      const uint64_t roomy = in_set + 2 * worst;
      rc = grow(D, b, a, roomy <= (1ull << 31) ? roomy : in_set + worst + worst / 4 + 65536, (uint32_t)tail0);
      if (rc) return rc;
      a.first = first;
      a.count = count;
      // the level's room in cells; the listed cells are committed with k + 1
      // insertions each, and each processed cell gives back what it did not
      // insert, so `committed` ends as the number of cells the level inserted
      a.room = (uint32_t)(b.cap - in_set);
      const uint32_t zero = 0, committed = count * (uint32_t)(k + 1);
      if (hipMemcpyAsync(&b.cnt->next, &zero, sizeof zero, hipMemcpyHostToDevice, D->stream) != hipSuccess ||
          hipMemcpyAsync(&b.cnt->committed, &committed, sizeof committed, hipMemcpyHostToDevice, D->stream) !=
              hipSuccess)
        return BDEG_E_DEVICE;
      rc = launch_pivot(D->stream, a, k, blocks);
      if (rc) return rc;
      if (hipMemcpyAsync(&c, b.cnt, sizeof c, hipMemcpyDeviceToHost, D->stream) != hipSuccess ||
          hipStreamSynchronize(D->stream) != hipSuccess)
        return BDEG_E_DEVICE;
      if (c.flags & PIVOT_ERR_STATE) return BDEG_E_ARG; // the start is not a lower facet
      if (c.flags & PIVOT_ERR_FULL) {
        regrow = true;
        break;
      }
      if (c.flags & PIVOT_TIE) {
        out.tie = true;
        return BDEG_OK;
      }
      if (c.committed < c.tail - tail0 || c.committed > a.room) return BDEG_E_DEVICE; // (room accounting)
      in_set += c.committed;
      first += count;
      count = c.tail - first;
    }
    if (regrow) {
      room = std::max(room, b.cap);
      continue;
    }
    out.tie = false;
    out.nvol = ((u128)c.vol_hi << 64) | c.vol_lo;
    out.cells = c.cells;
    if (cells_out) { // every cell is in the hash set (cells reached by pivots skip the list)
      std::vector<uint64_t> slots(2 * b.cap);
      if (hipMemcpy(slots.data(), b.table, slots.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return BDEG_E_DEVICE;
      cells_out->clear();
      for (uint64_t m : slots)
        if (m) cells_out->push_back(m);
      if (normals) {
        normals->masks = *cells_out;
        const int rc2 = normals_device(D, b.pts, b.hts, N, k, *normals);
        if (rc2) return rc2;
      }
    }
    return BDEG_OK;
  }
}

bdeg_u128 u128_out(u128 v) { return bdeg_u128{(uint64_t)v, (uint64_t)(v >> 64)}; }

} // namespace
} // namespace bdeg

using namespace bdeg;

extern "C" {

// Arguments of the walk's point-set entry points: shape, |h| < 2^40, the
// device width certificate, and a start mask of k + 1 points (0: Extend).
static int check_walk_points(const int32_t *points, const int64_t *heights, int N, int k, uint64_t start_mask) {
  if (!points || !heights || k < 1 || k > PIVOT_MAX_K || N < k + 1 || N > 64) return BDEG_E_ARG;
  if (start_mask != 0 && (__builtin_popcountll(start_mask) != k + 1 || (N < 64 && (start_mask >> N) != 0)))
    return BDEG_E_ARG;
  int64_t hmin = heights[0], hmax = heights[0];
  for (int j = 0; j < N; j++) {
    if (heights[j] >= (1ll << 40) || heights[j] <= -(1ll << 40)) return BDEG_E_ARG;
    hmin = std::min(hmin, heights[j]);
    hmax = std::max(hmax, heights[j]);
  }
  if (!device_bounds_ok(points, N, k, (uint64_t)(hmax - hmin))) return BDEG_E_OVERFLOW;
  return BDEG_OK;
}

int bdeg_pivot_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t start_mask,
                      uint64_t cap, uint64_t *cell_masks, uint64_t *n_cells, bdeg_u128 *nvol, int32_t *tie) {
  if (!n_cells || !nvol || !tie || (cap > 0 && !cell_masks)) return BDEG_E_ARG;
  int rc = check_walk_points(points, heights, N, k, start_mask);
  if (rc) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  std::vector<uint64_t> cells;
  WalkResult r;
  rc = walk(D, points, heights, N, k, start_mask, cap > 0 ? &cells : nullptr, r);
  if (rc) return rc;
  *tie = r.tie ? 1 : 0;
  *nvol = u128_out(r.nvol);
  *n_cells = r.tie ? 0 : r.cells;
  if (cap > 0 && !r.tie) memcpy(cell_masks, cells.data(), std::min<uint64_t>(cap, cells.size()) * sizeof(uint64_t));
  return BDEG_OK;
}

int bdeg_pivot_cells(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t start_mask,
                     uint64_t cap, uint64_t *cell_masks, int64_t *normal_num, uint64_t *normal_den,
                     uint64_t *n_cells, bdeg_u128 *nvol, int32_t *tie) {
  if (!n_cells || !nvol || !tie || (cap > 0 && (!cell_masks || !normal_num || !normal_den))) return BDEG_E_ARG;
  int rc = check_walk_points(points, heights, N, k, start_mask);
  if (rc) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  CellNormals cn;
  WalkResult r;
  rc = walk(D, points, heights, N, k, start_mask, nullptr, r, &cn);
  if (rc) return rc;
  *tie = r.tie ? 1 : 0;
  *nvol = u128_out(r.nvol);
  *n_cells = r.tie ? 0 : r.cells;
  if (r.tie || cap == 0) return BDEG_OK;
  if (cn.masks.size() != r.cells) return BDEG_E_STATE; // every processed cell is in the set exactly once
  const uint64_t n = std::min<uint64_t>(cap, cn.masks.size());
  memcpy(cell_masks, cn.masks.data(), n * sizeof(uint64_t));
  memcpy(normal_num, cn.num.data(), n * (size_t)k * sizeof(int64_t));
  memcpy(normal_den, cn.den.data(), n * sizeof(uint64_t));
  return BDEG_OK;
}

int bdeg_extend_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t *facet_mask,
                       int32_t *tie) {
  if (!facet_mask || !tie) return BDEG_E_ARG;
  int rc = check_walk_points(points, heights, N, k, 0);
  if (rc) return rc;
  int st;
  Device *D = device_get(&st);
  if (!D) return st;
  std::lock_guard<std::mutex> lk(D->mu);
  int32_t *d_pts = nullptr;
  int64_t *d_hts = nullptr;
  if (hipMalloc((void **)&d_pts, (size_t)N * k * sizeof(int32_t)) != hipSuccess ||
      hipMalloc((void **)&d_hts, (size_t)N * sizeof(int64_t)) != hipSuccess)
    rc = BDEG_E_NOMEM;
  if (!rc && (hipMemcpy(d_pts, points, (size_t)N * k * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
              hipMemcpy(d_hts, heights, (size_t)N * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess))
    rc = BDEG_E_DEVICE;
  uint64_t mask = 0;
  bool t = false;
  if (!rc) rc = extend_device(D, d_pts, d_hts, N, k, &mask, &t);
  if (d_pts) (void)hipFree(d_pts);
  if (d_hts) (void)hipFree(d_hts);
  if (rc) return rc;
  *facet_mask = t ? 0 : mask;
  *tie = t ? 1 : 0;
  return BDEG_OK;
}

int bdeg_degree_pivot(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits, bdeg_result *out) {
  if (!A || !out) return BDEG_E_ARG;
  memset(out, 0, sizeof *out);
  if (m < 1 || n < 1 || n > BDEG_MAX_N || lift_bits < 2 || lift_bits > 30) return out->status = BDEG_E_ARG;
  KernelPoints kp = kernel_points(A, m, n);
  if (kp.status != BDEG_OK) return out->status = kp.status;
  out->k = kp.k;
  out->rank = kp.rank;
  out->flags = kp.flags;
  out->components = u128_out(kp.comps);
  if (kp.k == 0) {
    out->nvol = bdeg_u128{1, 0};
    return out->status = BDEG_OK;
  }
  const int N = n + 1, k = kp.k;
  if (k > PIVOT_MAX_K) return out->status = BDEG_E_TOO_LARGE;
  out->candidates = binom_u64(N, k + 1);
  if (!device_bounds_ok(kp.pts.data(), N, k, (1ull << lift_bits) - 1)) return out->status = BDEG_E_OVERFLOW;
  int st;
  Device *D = device_get(&st);
  if (!D) return out->status = st;
  std::lock_guard<std::mutex> lk(D->mu);
  std::vector<int64_t> h(N);
  for (int attempt = 0; attempt < BDEG_MAX_ATTEMPTS; attempt++) {
    // the lifting bdeg_degree draws for the same seed (single-system stream)
    const uint64_t key = lift_key(seed, 0, (uint32_t)attempt);
    for (int j = 0; j < N; j++) h[j] = lift_height(key, j, lift_bits);
    WalkResult r;
    const int rc = walk(D, kp.pts.data(), h.data(), N, k, 0, nullptr, r);
    out->attempts = attempt + 1;
    if (rc) return out->status = rc;
    if (r.tie) continue;
    out->nvol = u128_out(r.nvol);
    out->cells = r.cells;
    return out->status = BDEG_OK;
  }
  return out->status = BDEG_E_TIE;
}

} // extern "C"
