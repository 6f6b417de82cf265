// Internal structures shared by the host runtime and the HIP kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bdeg.h"
#include "lifting.hpp"

namespace bdeg {

typedef unsigned __int128 u128;
typedef __int128 i128;

// Per-system device descriptor.  Points are int32 (k coordinates each),
// heights int64; both live in flat device arrays at the given offsets.
struct SysDesc {
  int32_t N;         // points (n + 1), N <= 64
  int32_t k;         // spatial dimension
  int32_t pt_off;    // first int32 of the N x k points
  int32_t ht_off;    // first int64 of the N heights
  int32_t lift_bits; // heights uniform in [0, 2^lift_bits)
  int32_t npad_log2; // lanes per point group: 8, 16, 32 or 64
  uint64_t lift_key; // counter-based lifting key for the current attempt
  uint64_t seed;      // the system's lifting stream is (seed, sys_index, attempt)
  uint32_t sys_index; // stream index: 0 for every seeded system (one-shot, batch and served alike)
  uint32_t flags;     // SYS_DENSE, SYS_SORTED
};

// A work unit: the candidates whose top elements (colex) are exactly the set
// bits of `mask` and whose remaining elements lie below the lowest set bit,
// with the next element restricted to [c_lo, c_hi] (a run of sibling
// subtrees; 0 and 63 when unrestricted).
struct Tile {
  uint64_t mask;
  uint32_t sys;
  uint8_t c_lo, c_hi;
  uint16_t pad;
};
// host-side work unit with its candidate count (for ordering)
struct TileC {
  Tile t;
  uint64_t cost;
};

// Per-system device accumulators (sum of |det| of lower facets, as a 128-bit
// value in two 64-bit words, cell count and the tie flag).
struct SysAcc {
  uint64_t lo, hi;
  uint64_t cells;
  uint32_t tie;
  uint32_t attempt; // lifting draws made on the device beyond the host's (in-pass redraws)
};

// Device-wide counters (zeroed per run).
struct DevCounters {
  uint64_t ridges, inner, sp_upd, pruned, leaves, tiles;
  uint64_t rsteps, lsteps, lempty; // wavefront loop iterations (ridge, leaf, leaf without candidates)
  // the same work weighted by the points it touches (exact over systems of
  // different N): N * inner, N * sp_upd, N * ridges, (N - k - 1) * leaves
  uint64_t w_inner, w_spatial, w_ridges, w_leaves;
  // lane-dense kernel: candidates set up (with or without D = 0), the units
  // it ran, and the candidates among the first set up as tail quadruples
  uint64_t triples, dunits, quads;
  uint32_t next_tile; // dynamic work queue head
  uint32_t error;     // a work unit exceeded its step budget (watchdog)
};

// ------------------------------------------------------------ host algebra
struct KernelPoints {
  int status = BDEG_OK;
  int k = 0, rank = 0, m = 0, n = 0;
  u128 comps = 0;
  uint32_t flags = 0;
  std::vector<int32_t> pts; // (n+1) x k, point 0 = origin
};
KernelPoints kernel_points(const int64_t *A, int m, int n);

// Device certification: every Bareiss quantity of the device path fits the
// narrow types (spatial minors int32, height minors int64, products in 96 bits).
// `height_span` is max(h) - min(h) over the points.  Every spatial minor is
// below 2^spatial_bits and every height minor below 2^height_bits (Hadamard).
bool device_bounds_ok(const int32_t *pts, int N, int k, uint64_t height_span, int spatial_bits = 31,
                      int height_bits = 60);
// The lane-dense kernel (enum_dense.hpp) needs k >= 3, spatial minors
// < 2^30 and height minors < 2^59; false also when the process asked for the
// lanes-as-points schedule everywhere (bdeg_set_schedule).
bool dense_ok(const int32_t *pts, int N, int k, uint64_t height_span);
constexpr uint32_t SYS_DENSE = 1; // SysDesc.flags: units run in the lane-dense kernel
// SysDesc.flags: the units cover every candidate of the system, so the
// lane-dense kernel may relabel its points (it orders them by lifted height)
constexpr uint32_t SYS_SORTED = 2;

// ------------------------------------------------------------ tiling
uint64_t binom_u64(int n, int r); // saturates at UINT64_MAX
// Cover all (k+1)-subsets of N points with subtrees of at most `max_cost`
// candidates where possible (never deeper than k points chosen).
void tiles_full(int N, int k, uint32_t sys, uint64_t max_cost, std::vector<TileC> &out);
// Exactly the candidates with colex rank in [lo, hi).
// Subtrees fully inside the range are further split down to max_cost.
void tiles_range(int N, int k, uint32_t sys, uint64_t lo, uint64_t hi, uint64_t max_cost, std::vector<TileC> &out);
// colex rank interval [start, end) covered by a unit
void tile_interval(const Tile &t, int k, uint64_t *start, uint64_t *end);
// order work units by decreasing cost and strip the costs
void tiles_sorted(std::vector<TileC> &in, std::vector<Tile> &out);


// Device cell list: vertex masks of lower facets, appended through `count`
// (facets beyond `cap` are counted, not stored).
struct CellSink {
  uint64_t *masks;
  uint64_t cap;
  uint64_t *count;
};

// ------------------------------------------------------------ cell walk (kernels_pivot*.hip)
constexpr int PIVOT_MAX_K = BDEG_PIVOT_MAX_K; // deepest k of the cell walk
constexpr int PIVOT_DFS_MAX = 32;              // cells reached by pivots from one claimed cell, at most
constexpr int PIVOT_CREDIT_CELLS = 64;         // a wave takes the level's room in chunks of this many cells
constexpr int PIVOT_CLAIM_BATCH = 16;          // listed cells a wave claims at once in wide levels
constexpr int PIVOT_SWAPS = 6;                 // points two claimed cells may differ in for pivots between them
constexpr uint32_t PIVOT_TIE = 1;       // a non-generic lower face was met
constexpr uint32_t PIVOT_ERR_FULL = 2;  // hash set or work list out of room
constexpr uint32_t PIVOT_ERR_STATE = 4; // a listed cell is not a lower facet (bad start cell)

struct PivotCounters {
  uint32_t next;  // work item head of the current level
  uint32_t tail;  // cells in the work list
  uint32_t flags; // PIVOT_*
  uint32_t pad;
  unsigned long long vol_lo, vol_hi; // sum of |D| over processed cells (128-bit)
  unsigned long long cells;          // processed cells
  uint32_t committed; // the level's insertions, plus k + 1 per committed cell not yet processed
  uint32_t pad2;
};

struct PivotArgs {
  const int32_t *pts; // N x k
  const int64_t *hts; // N
  int N;
  uint64_t *list;     // work list of cells (vertex masks), in discovery order
  uint32_t first;     // this level's cells are list[first, first + count)
  uint32_t count;
  uint32_t cap_list;
  uint64_t *table;    // hash set of cells (0 = empty), power-of-two size
  uint64_t table_mask;
  uint32_t room;      // cells the set and the list can take in this level (bounds `committed`)
  PivotCounters *cnt;
};
typedef void (*PivotFn)(PivotArgs);
// One level of the walk: every cell of [first, first + count) is processed by
// one wavefront of a persistent grid of `blocks` blocks of 4 wavefronts.
int launch_pivot(void *stream, const PivotArgs &a, int k, int blocks);
int max_pivot_blocks(int k);
// Insert the nonzero entries of old[0, n_old) (the previous set) into the
// (cleared) hash set a.table.
int launch_pivot_rehash(void *stream, const PivotArgs &a, const uint64_t *old, uint64_t n_old);

// ------------------------------------------------------------ Extend (kernels_extend.hip)
constexpr uint32_t EXTEND_TIE = 1;       // a lower face is not a simplex (the lifting is not generic)
constexpr uint32_t EXTEND_ERR_SPAN = 2;  // the points do not span the space affinely
constexpr uint32_t EXTEND_ERR_RANGE = 4; // an exact division failed (outside the certified widths)
struct ExtendResult {
  uint64_t mask; // the lower facet found (k + 1 points), 0 on failure
  uint32_t flags;
  uint32_t pad;
};
// One wavefront: a lower facet of the lifted points by exact supporting-
// hyperplane rotations from the lowest point (N <= 64, k <= PIVOT_MAX_K).
int launch_extend(void *stream, const int32_t *d_pts, const int64_t *d_hts, int N, int k, ExtendResult *d_out);

// ------------------------------------------------------------ prefix pruning (kernels_prune.hip)
constexpr int PRUNE_WMAX = 8; // widest prefix state tested (free spatial columns)
struct PruneCounters {
  uint32_t next;             // item head
  uint32_t units;            // work units emitted
  uint32_t degenerate;       // prefixes whose points are affinely dependent
  uint32_t pruned;           // prefixes certified to lie in no lower face
  unsigned long long pivots; // simplex pivots of all tests
  uint32_t overflow;         // the unit buffer was too small
  uint32_t pad;
};
struct PruneArgs {
  const int32_t *pts; // N x K
  const int64_t *hts; // N
  int N, K, W;        // W = K + 1 - |prefix|
  const uint64_t *items;
  uint32_t n_items;   // prefixes (vertex masks), all with K + 1 - W points
  Tile *units;        // out: for each prefix F kept and next element c, the units
  uint32_t cap_units; //   (F + c, run) for the runs of chunk c, in bucket c:
  const uint32_t *bucket_off; // units[bucket_off[c] + (running count)]
  uint32_t *bucket_cnt;
  const uint16_t *chunk_start; // chunk c: runs chunk_start[c] .. chunk_start[c + 1] - 1
  const uint8_t *run_lo, *run_hi; // run [run_lo, run_hi] of the element after c
  PruneCounters *cnt;
};
// One wavefront per prefix: eliminate it, test it, emit the units below it.
int launch_prune(void *stream, const PruneArgs &a);
// Gather buckets c_hi .. c_lo of the bucketed units into one list (in order).
int launch_prune_compact(void *stream, const Tile *in, Tile *out, const uint32_t *off, const uint32_t *cnt, int c_lo,
                         int c_hi, uint32_t cap);

// ------------------------------------------------------------ kernels (kernels.hip)
// enumeration kernel variants
constexpr int MODE_PLAIN = 0; // volume, cell count and tie flag
constexpr int MODE_STATS = 1; // also count the work (profiling)
constexpr int MODE_EMIT = 2;  // also list every lower facet (single-k kernels only)

// host-side handle of one enumeration kernel instantiation
// rerun (optional): rerun[0] != 0 when some system is redrawn in this pass,
// rerun[1 + s] != 0 for the systems whose units are run (the others' units are
// skipped); nullptr runs every unit.
typedef void (*EnumFn)(const SysDesc *, const int32_t *, const int64_t *, const Tile *, uint32_t, SysAcc *,
                       DevCounters *, CellSink, const uint32_t *);

struct LaunchShape {
  int blocks = 0;
  int waves_per_block = 4;
  bool single = false; // every unit launched has N > 32 points: one point group per wavefront
  bool dense = false;  // every unit launched belongs to a SYS_DENSE system: the lane-dense kernel
  int mode = MODE_PLAIN;
  CellSink sink{nullptr, 0, nullptr}; // MODE_EMIT only
  const uint32_t *rerun = nullptr;    // in-pass redraw round: gate and per-system flags
};
// point groups per wavefront for N points: 64 / (smallest power of two >= N, at least 8)
inline int groups_for(int N) { return N <= 8 ? 8 : N <= 16 ? 4 : N <= 32 ? 2 : 1; }
// units of systems with one point group per wavefront run in their own kernel variant
inline bool single_group(int N) { return groups_for(N) == 1; }
inline int npad_log2_for(int N) { return N <= 8 ? 3 : N <= 16 ? 4 : N <= 32 ? 5 : 6; }
// Launch helpers; all asynchronous on `stream` (a hipStream_t).
int launch_lift(void *stream, const SysDesc *d_sys, const int32_t *d_active, int n_active,
                int64_t *d_heights);
int launch_clear(void *stream, SysAcc *d_acc, int n_sys, DevCounters *d_cnt, int n_cnt);
int launch_clear_list(void *stream, SysAcc *d_acc, const int32_t *d_list, int n);
// Start of a replayable seeded pass: every system back to attempt 0 (lifting
// key, cleared sums), counter blocks and redraw gates cleared.
int launch_reset(void *stream, SysDesc *d_sys, SysAcc *d_acc, int n_sys, DevCounters *d_cnt, int n_cnt,
                 uint32_t *d_rerun, int rounds);
// One in-pass redraw round: every system whose sums report a tie (and has
// draws left) gets attempt + 1, a new lifting and cleared sums, and is marked
// in rerun[1 + s]; rerun[0] is set when any is.
int launch_retie(void *stream, SysDesc *d_sys, SysAcc *d_acc, int64_t *d_heights, int n_sys, uint32_t *d_rerun);
int launch_enumerate(void *stream, const SysDesc *d_sys, const int32_t *d_pts,
                     const int64_t *d_heights, const Tile *d_tiles, uint32_t n_tiles, SysAcc *d_acc,
                     DevCounters *d_cnt, int kmin, int kmax, LaunchShape shape);
int device_cu_count();
// Inner normals of listed lower facets (one thread per facet): for the facet
// with vertex mask masks[i] of the N x k points (int32) and heights, num[i*k ..]
// and den[i] > 0 with alpha = num / den; sets *d_err on a malformed mask or
// a value outside int64.
int launch_cell_normals(void *stream, const uint64_t *d_masks, uint64_t n, const int32_t *d_pts,
                        const int64_t *d_hts, int N, int k, int64_t *d_num, uint64_t *d_den, uint32_t *d_err);
int max_enum_blocks(int kmin, int kmax, int waves_per_block, bool single,
                    bool dense = false); // occupancy-derived persistent grid

} // namespace bdeg
