/*
 * bdeg -- exact degree of the C*-solution set of a binomial system x^A = b
 * on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2 of Chen & Mehta, "Parallel degree computation for
 * solution space of binomial systems"): a system of m binomial equations
 * c1 x^alpha + c2 x^beta = 0 in n variables is x^A = b with A the integer
 * exponent matrix.  HERE A IS m x n, ROW-MAJOR, ONE ROW PER BINOMIAL
 * (row i = alpha^(i) - beta^(i)); the paper writes the transpose.
 *
 * For a consistent system the library returns, exactly:
 *   k          = n - rank(A), the dimension of every component;
 *   components = |d_1 ... d_r|, the product of the nonzero Smith invariant
 *                factors (Proposition "topological"): the number of components;
 *   nvol       = k! Vol_k(conv{0, v_1, ..., v_n}) where v_i is row i of a
 *                saturated integer basis V (n x k) of ker(A): the degree of
 *                each component (Proposition "degree", eq. "deg-vol").
 * The degree of the whole solution set is components * nvol.
 *
 * nvol is computed on the GPU as the sum of |det| over the lower facets of a
 * generic integer lifting of the points (Section 4, eqs. "lower-face" and
 * "simplex-vol"): every candidate (k+1)-subset is decided exactly in integer
 * arithmetic.  A lifting that produces a non-simplicial lower face (a "tie")
 * is redrawn; the result never depends on the seed, only `attempts` does.
 *
 * Conventions shared by every entry point
 *   - All pointers are HOST pointers unless stated; the caller owns every
 *     buffer, the library copies inputs and keeps no caller pointer.
 *   - Integers are little-endian; 128-bit results are {lo, hi} words.
 *   - Return value: BDEG_OK (0) or a negative BDEG_E_* code; bdeg_strerror
 *     gives a message.  On error the outputs are left in an unspecified state
 *     unless stated.
 *   - Thread safety: calls may come from several host threads; the library
 *     serialises device work on its own stream per process.
 *   - The device is the process's current HIP device at the first call
 *     (or the one given to bdeg_init).  No GPU => BDEG_E_DEVICE.
 */
#ifndef BDEG_H
#define BDEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDEG_OK 0
#define BDEG_PENDING 1        /* serving: the request is not finished yet */
#define BDEG_E_ARG (-1)       /* null pointer, bad size, bad lifting width */
#define BDEG_E_OVERFLOW (-2)  /* host int64 algebra overflowed, or the point set's minor bounds
                                 exceed what the exact device arithmetic certifies */
#define BDEG_E_TOO_LARGE (-3) /* k > BDEG_MAX_K, or more than 2^63 candidates */
#define BDEG_E_TIE (-4)       /* no generic lifting found in BDEG_MAX_ATTEMPTS draws */
#define BDEG_E_DEVICE (-5)    /* HIP runtime error or no device */
#define BDEG_E_NOMEM (-6)     /* device or host allocation failed / over budget */
#define BDEG_E_STATE (-7)     /* unknown ticket, closed server, or result already taken */

#define BDEG_F_NEEDS_CONSISTENCY 1u /* rank < m: the set is empty unless b^(Q_0) = 1
                                       (Section 2, eq. "consistency"); b is not an input */
#define BDEG_F_PRUNED 2u            /* the volume came from the prefix-pruned enumeration
                                       (see bdeg_degree; the same value either way) */

#define BDEG_MAX_N 63        /* variables: N = n + 1 points fit one 64-lane wavefront */
#define BDEG_MAX_K 18        /* kernel dimension handled on the device */
#define BDEG_MAX_ATTEMPTS 16 /* lifting draws before BDEG_E_TIE */

typedef struct {
  uint64_t lo, hi;
} bdeg_u128;

/* Result of one system.  Beyond the three numbers the method defines (k,
 * components, nvol) it reports what callers of batches and liftings need:
 * a per-system status, the rank, the lifting draws used, the consistency
 * flag, the candidates decided and the cells of the final lifting; the
 * `reserved` word keeps the 128-bit fields 16-byte aligned.  Likewise every
 * entry point that draws a lifting takes its height width `lift_bits` beside
 * the seed (the results do not depend on either; only `attempts` does). */
typedef struct {
  int32_t status;       /* BDEG_OK or a BDEG_E_* code for this system */
  int32_t k;            /* n - rank(A) */
  int32_t rank;         /* r */
  int32_t attempts;     /* lifting draws used (1 + tie retries); 0 when k == 0 */
  uint32_t flags;       /* BDEG_F_* */
  uint32_t reserved;
  bdeg_u128 components; /* |prod of nonzero Smith invariant factors| */
  bdeg_u128 nvol;       /* k! Vol_k(conv{0, v_1..v_n}); 1 when k == 0 */
  uint64_t candidates;  /* C(n+1, k+1): candidate simplices decided */
  uint64_t cells;       /* lower facets of the final lifting (cells of the subdivision) */
} bdeg_result;

/* Device work counters of the last device run (for roofline accounting). */
typedef struct {
  uint64_t ridges;            /* subtree nodes with k points fixed (each tests its candidates) */
  uint64_t inner_nodes;       /* subtree nodes with 2..k-1 points fixed */
  uint64_t spatial_updates;   /* spatial residual columns eliminated over all inner nodes */
  uint64_t pruned;            /* prefixes cut because the new point is affinely dependent */
  uint64_t leaves;            /* candidates tested with a nonzero determinant */
  uint64_t tiles;             /* work units processed */
  uint64_t ridge_steps;       /* wavefront iterations of the ridge loops (one ridge per lane group) */
  uint64_t leaf_steps;        /* wavefront iterations of the leaf loops (one candidate per lane group) */
  uint64_t empty_steps;       /* leaf iterations in which no lane group had a candidate with D != 0 */
  /* the same work weighted by the points each step touches, summed over the
     systems (exact for batches of mixed N and k): */
  uint64_t point_inner;       /* sum of N * inner_nodes */
  uint64_t point_spatial;     /* sum of N * spatial_updates */
  uint64_t point_ridges;      /* sum of N * ridges */
  uint64_t leaf_points;       /* points the leaf tests examined: (N - k - 1) per leaf with lanes
                                 as points; in the lane-dense kernel, per candidate, the points up to
                                 its first point proved below (its test batch may stop there), or
                                 N - k - 1 */
  /* lane-dense schedule (BDEG_SCHED_AUTO): it creates no ridges; there
     `ridges` counts its nodes with three spatial columns left, `leaves` the
     candidates with D != 0 it tested, ridge_steps its setup passes,
     leaf_steps its test batches and empty_steps the candidates with no
     point proved below them by the batch test, decided one by one with
     lanes as points (the cells, the ties, and candidates whose points below
     all lie within the test's band) */
  uint64_t triples;           /* candidates it set up (any D): triples of nodes with three
                                 spatial columns left and tail quadruples */
  uint64_t dense_units;       /* work units run by the lane-dense kernel */
  uint64_t quads;             /* the tail quadruples among `triples` (set up from nodes with
                                 four spatial columns left) */
  float kernel_ms;            /* device time of the enumeration kernel, HIP events */
  float total_ms;             /* device time of the whole device pass (clear, lift, enumerate) */
  int32_t captured;           /* 1: the device pass replays captured HIP graphs; 0: plain launches */
  int32_t redraws;            /* systems whose tied lifting was redrawn inside the last device pass */
} bdeg_stats;

/* Enumeration schedule for the whole process (default BDEG_SCHED_AUTO).
 * Both decide every candidate exactly and give identical results; they differ
 * in how a wavefront's lanes are used.
 *   BDEG_SCHED_AUTO    systems with k >= 3 whose minors the host certifies
 *                      below 2^30 (spatial) and 2^59 (with heights) run in
 *                      the lane-dense kernel: the depth-first walk stops with
 *                      three spatial columns left, and each lane then tests a
 *                      whole candidate against every point (cofactors by
 *                      Sylvester's identity); all other systems as below.
 *   BDEG_SCHED_POINTS  every system in the lanes-as-points kernel: lane j
 *                      holds point j down to single candidates.
 * Returns BDEG_E_ARG for another value.  Takes effect for work planned after
 * the call (prepared batches keep the schedule they were created with). */
#define BDEG_SCHED_AUTO 0
#define BDEG_SCHED_POINTS 1
int bdeg_set_schedule(int32_t schedule);

/* Optional: select the HIP device (default: current device at first use).
 * Must precede every other call; BDEG_E_STATE if the library is already set up. */
int bdeg_init(int32_t device);

/*
 * Degree data of one binomial system (Sections 2-4).
 *   A          m x n row-major int64 exponent matrix, 1 <= m, 1 <= n <= BDEG_MAX_N.
 *   seed       selects the lifting stream (results do not depend on it).
 *   lift_bits  heights uniform in [0, 2^lift_bits), 2 <= lift_bits <= 30.
 *   out        filled on BDEG_OK; out->status repeats the return code.
 * Cost model: under BDEG_SCHED_AUTO a system of at least
 * BDEG_PRUNE_MIN_CANDIDATES candidate (k+1)-subsets is enumerated with
 * prefix pruning (bdeg_nvol_points_pruned on the same seeded heights, ties
 * redrawn the same way; out->flags gets BDEG_F_PRUNED).  The result is the
 * same, attempts and cells included; below that size the pruning filter
 * costs more than it saves (measured: 0.67 against 0.42 ms at 1.0e7
 * candidates, 7.7 against 14.8 ms at 8.5e8).  bdeg_degree_batch applies the
 * same rule per system; prepared batches and the server do not prune.
 */
#define BDEG_PRUNE_MIN_CANDIDATES (1ull << 27)
int bdeg_degree(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits,
                bdeg_result *out);

/*
 * Many systems in one device launch (continuous tile queue over all systems).
 *   A_concat   the matrices back to back, system s is m[s] x n[s] row-major.
 *   m, n       count entries each.  out: count results (per-system status).
 * Returns BDEG_OK if every system succeeded, else the first failing code
 * (every out[s].status is still filled).  Each system draws its liftings from
 * the same stream as a one-shot bdeg_degree call with this seed, so out[s]
 * equals bdeg_degree's result for system s, attempts and cells included.
 */
int bdeg_degree_batch(const int64_t *A_concat, const int32_t *m, const int32_t *n, int32_t count,
                      uint64_t seed, int32_t lift_bits, bdeg_result *out);

/*
 * Prepared batch: host algebra done once, point sets and work lists resident
 * in device memory, device path captured as a HIP graph and replayable.
 *   bdeg_batch_create   host prologue (Smith form, kernel points, bounds,
 *                       tiling) + upload; *out owns device memory.
 *   bdeg_batch_run      enqueue one full device pass on the library stream
 *                       (async): reset to the first lifting, enumeration, then
 *                       up to 3 redraw rounds in which every tied system gets
 *                       its next lifting and its units run again (a round
 *                       with no tie costs one empty launch).  The pass is
 *                       three captured HIP graphs (bdeg_stats.captured).
 *   bdeg_batch_results  wait; a system still tied after the captured rounds
 *                       is redrawn by uncaptured reruns until it is not (at
 *                       most BDEG_MAX_ATTEMPTS draws in all); fill out[count].
 *                       Results equal bdeg_degree's for the same seed and
 *                       lift_bits, attempts included.
 *   bdeg_batch_stats    HIP-event times of the last run, and the work counters
 *                       of the last profiling pass.
 *   bdeg_batch_profile  one extra synchronous device pass with the kernel
 *                       variant that also counts its work (same lifting, same
 *                       work); fills the counters of bdeg_batch_stats.
 *   bdeg_batch_destroy  free everything.
 */
typedef struct bdeg_batch bdeg_batch;
int bdeg_batch_create(const int64_t *A_concat, const int32_t *m, const int32_t *n, int32_t count,
                      uint64_t seed, int32_t lift_bits, bdeg_batch **out);
int bdeg_batch_run(bdeg_batch *b);
int bdeg_batch_results(bdeg_batch *b, bdeg_result *out);
int bdeg_batch_stats(const bdeg_batch *b, bdeg_stats *out);
int bdeg_batch_profile(bdeg_batch *b);
int bdeg_batch_destroy(bdeg_batch *b);

/*
 * Autotuner of a prepared batch's work schedule.  The systems are grouped in
 * buckets of equal k and equal smallest lane-group width (8, 16, 32 or 64
 * lanes per point group for N <= 8, 16, 32, 64 points).  For each bucket the
 * bucket's systems are enumerated alone under every schedule of a small grid
 * (the kernel: lanes as points -- a point per lane, at the smallest or the
 * next larger lane-group width, 64 lanes meaning one group per wavefront in
 * its own kernel variant -- or lane-dense, a candidate per lane, for the
 * systems it is certified for; work-unit size cap: 128 .. 8192 candidates)
 * and under the default schedule, each timed by HIP events (median of `reps`
 * passes after a warm-up).  Every schedule must give
 * exactly the default's sums for every system (the same liftings and
 * candidates), else BDEG_E_STATE and nothing is written.  The fastest
 * schedule per bucket is written to the JSON table `table_path` (entries of
 * buckets the batch lacks are kept; NULL: not written) and applied to the
 * batch, whose device pass is captured again.
 * bdeg_batch_create applies the table named by the environment variable
 * BDEG_TUNE_TABLE, else tuning/gfx950.json beside the library, when it
 * exists; a system of a bucket without an entry keeps the default schedule.
 * The paper tunes its thread counts by hand (Section 6, Table 5); this
 * replaces that with a measured choice per bucket.
 */
int bdeg_batch_tune(bdeg_batch *b, const char *table_path, int32_t reps);

/*
 * Volume of a caller's point set with caller's heights, restricted to the
 * candidates whose colex rank lies in [rank_lo, rank_hi)
 * (rank {c_0 < ... < c_k} = sum_i C(c_i, i+1); pass rank_hi = UINT64_MAX for
 * all).  No tie retry: *tie reports a non-generic lower face in the range.
 *   points   N x k row-major int32 (N <= 64, 1 <= k <= BDEG_MAX_K);
 *   heights  N int64, |h| < 2^40.
 * The point set must satisfy the device bound (see BDEG_E_OVERFLOW).
 */
int bdeg_nvol_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k,
                     uint64_t rank_lo, uint64_t rank_hi, bdeg_u128 *nvol, int32_t *tie,
                     uint64_t *cells);

/*
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): exactly
 * bdeg_nvol_points (same arguments, results and errors), with every device
 * buffer it uses -- the staged points and heights, the work units, the
 * accumulator and the counters -- carved from one static device array of
 * BDEG_NOALLOC_SCRATCH_BYTES that each GPU holds until the process ends.  It
 * calls no hipMalloc or hipFree and no allocating device library routine
 * (the host side of the plan reuses its buffers across calls).
 *   Limit: at most BDEG_NOALLOC_MAX_UNITS work units.  The plan is coarsened
 *   (larger units) until it fits; BDEG_E_TOO_LARGE when even units of 2^26
 *   candidates are too many (more than about 8.8e12 candidates in the range).
 *   Sharing: every call on one GPU uses that GPU's array, which keeps the last
 *   call's contents (each call clears what must start at zero).  Calls through
 *   this library are serialised by its device lock; any other work that
 *   overlapped a call on the same array would race with it.
 */
#define BDEG_NOALLOC_MAX_UNITS (1 << 17)
#define BDEG_NOALLOC_SCRATCH_BYTES ((size_t)BDEG_NOALLOC_MAX_UNITS * 16u + 32768u)
int bdeg_nvol_points_noalloc(const int32_t *points, const int64_t *heights, int32_t N, int32_t k,
                             uint64_t rank_lo, uint64_t rank_hi, bdeg_u128 *nvol, int32_t *tie,
                             uint64_t *cells);

/*
 * Cells of the regular subdivision (Section 4) with their inner normals:
 * the lower facets among the candidates whose colex rank lies in
 * [rank_lo, rank_hi), each with the unique inner normal (alpha, 1) of eq.
 * "lower-d-face-again", alpha = num / den exactly.  They are the start data
 * of the polyhedral homotopies of Section 5 (one homotopy per cell).
 *   points, heights, N, k, rank_lo, rank_hi  as for bdeg_nvol_points;
 *   cell_masks [cap]      bit i set for vertex i (the facet's k+1 points);
 *   normal_num [cap * k]  numerators of alpha, one row of k per cell;
 *   normal_den [cap]      den = the cell's normalized volume |D| > 0;
 *   *n_cells              the number of cells found; at most cap are written
 *                         (a larger count asks for a larger buffer; cap = 0
 *                         only counts, and the arrays may then be NULL);
 *   *tie                  as for bdeg_nvol_points (the list is then not a
 *                         subdivision).
 * Cells come in no particular order; den over all cells sums to the volume
 * bdeg_nvol_points gives.  Device memory for cap cells is allocated per call.
 * Errors: BDEG_E_ARG, BDEG_E_OVERFLOW (device bound, or a numerator outside
 * int64), BDEG_E_DEVICE, BDEG_E_NOMEM.
 */
int bdeg_cells_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k,
                      uint64_t rank_lo, uint64_t rank_hi, uint64_t cap, uint64_t *cell_masks,
                      int64_t *normal_num, uint64_t *normal_den, uint64_t *n_cells, int32_t *tie);

/*
 * The regular subdivision behind bdeg_degree: the same host prologue, seeded
 * lifting and tie retries, so *out equals bdeg_degree(A, m, n, seed,
 * lift_bits) and the cells' den sum to out->nvol.  Also returned: the point
 * set (points: room for (n+1)*n int32; (n+1)*k written, point 0 first), the
 * heights of the lifting that succeeded (heights: n+1 int64) and the cells
 * as for bdeg_cells_points (normal_num: room for cap*n int64; cap*k written).
 * k == 0 or an error: *n_cells = 0 and the status as for bdeg_degree.
 */
int bdeg_subdivision(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits,
                     uint64_t cap, int32_t *points, int64_t *heights, uint64_t *cell_masks,
                     int64_t *normal_num, uint64_t *normal_den, uint64_t *n_cells, bdeg_result *out);

/*
 * bdeg_nvol_points over all candidates, with prefix pruning (Section 4.1: a
 * set of points that is not a lower face extends to no lower facet).  The
 * candidates are split by their top d = k + 1 - W points; one wavefront per
 * such prefix decides, with a float simplex whose answer is then certified in
 * exact integer arithmetic, whether the prefix lies in a lower face, and only
 * the subtrees of prefixes that may are enumerated.  The results are those of
 * bdeg_nvol_points (a pruned subtree holds no lower facet and no tie).
 *   width      W, 1..8 free columns of the tested prefix states (0: 5, widened
 *              while there are more than 2^18 prefixes); BDEG_E_TOO_LARGE when
 *              the prefixes exceed BDEG_PRUNE_MAX_PREFIXES;
 *   *nvol, *tie, *cells   as for bdeg_nvol_points;
 *   stats      optional (NULL): prefixes, degenerate and pruned ones, units
 *              enumerated, simplex pivots, device times of both phases.
 */
#define BDEG_PRUNE_MAX_PREFIXES (1ull << 24)
typedef struct bdeg_prune_stats {
  uint64_t prefixes;   /* prefixes tested */
  uint64_t degenerate; /* prefixes whose points are affinely dependent (no candidate below) */
  uint64_t pruned;     /* prefixes certified to lie in no lower face */
  uint64_t units;      /* work units enumerated below the other prefixes */
  uint64_t pivots;     /* simplex pivots of all tests */
  int32_t prefix_size; /* d */
  int32_t width;       /* W = k + 1 - d */
  float filter_ms;     /* device time of the prefix tests */
  float enum_ms;       /* device time of the enumeration of the units kept */
} bdeg_prune_stats;
int bdeg_nvol_points_pruned(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, int32_t width,
                            bdeg_u128 *nvol, int32_t *tie, uint64_t *cells, bdeg_prune_stats *stats);

/*
 * The regular subdivision by simplicial pivoting (Section 4.2-4.4): instead
 * of deciding every (k+1)-subset, walk from one cell to its neighbours across
 * facets (for the facet opposite v, the new vertex minimizes the height above
 * the cell's hyperplane over the distance beyond the facet), keeping a device
 * hash set of visited cells.  The work follows the number of cells, so k up
 * to BDEG_PIVOT_MAX_K and N up to 64 are in reach when the cells are few.
 *   points, heights  as for bdeg_nvol_points (k <= BDEG_PIVOT_MAX_K);
 *   start_mask       a cell (k+1 points) that is a lower facet for `heights`
 *                    (BDEG_E_ARG when it is not), or 0: the start cell is
 *                    found by bdeg_extend_points' method on the device;
 *   cell_masks [cap] the cells, in no particular order (cap = 0: none copied);
 *   *n_cells, *nvol  number of cells and the sum of their normalized volumes;
 *   *tie             a non-generic lower face was met (results then invalid).
 * Device memory grows with the walk: before each breadth-first level the
 * work list (8 bytes per cell) and the hash set (16 bytes per cell) are
 * grown, by doubling, to the cells so far plus (k + 1) per cell of the level
 * (twice that while it fits); BDEG_E_NOMEM when that passes 2^31 cells.
 */
#define BDEG_PIVOT_MAX_K 24
int bdeg_pivot_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k,
                      uint64_t start_mask, uint64_t cap, uint64_t *cell_masks, uint64_t *n_cells,
                      bdeg_u128 *nvol, int32_t *tie);

/*
 * Degree data of x^A = b (as bdeg_degree) computed by the cell walk, for k up
 * to BDEG_PIVOT_MAX_K.  The lifting is bdeg_degree's seeded generic lifting
 * (the same heights for the same seed and lift_bits), the start cell comes
 * from Extend (bdeg_extend_points), and a tie redraws the lifting (at most
 * BDEG_MAX_ATTEMPTS draws).  For k <= BDEG_MAX_K the result equals
 * bdeg_degree's, cells and attempts included (the same regular subdivision).
 */
int bdeg_degree_pivot(const int64_t *A, int32_t m, int32_t n, uint64_t seed, int32_t lift_bits,
                      bdeg_result *out);

/*
 * Extend (Section 4.1, the lower-face LP of eq. "ext-lp"; Section 4.5,
 * algorithm Extend): a lower facet of the caller's lifted points, the start
 * of the walk.  From the lowest lifted point, the face is grown one point at
 * a time by tilting a supporting hyperplane of the current lower face about
 * it until the first other lifted point reaches it (an exact ratio test on
 * fraction-free residuals, one wavefront on the device); after k steps the
 * face is a lower facet.  Exact integer arithmetic throughout.
 *   points, heights  as for bdeg_pivot_points (k <= BDEG_PIVOT_MAX_K);
 *   *facet_mask      the k + 1 points of the facet (0 when *tie);
 *   *tie             1 when a lower face met on the way is not a simplex
 *                    (the lifting is not generic).
 * Errors: BDEG_E_ARG (bad sizes, heights |h| >= 2^40, points that do not span
 * Z^k affinely), BDEG_E_OVERFLOW (outside the device width certificate),
 * BDEG_E_DEVICE, BDEG_E_NOMEM.
 */
int bdeg_extend_points(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t *facet_mask,
                       int32_t *tie);

/*
 * The cell walk (as bdeg_pivot_points; start_mask 0 = Extend) returning the
 * cells with their inner normals (alpha, 1) of eq. "lower-d-face-again",
 * alpha = num / den exactly, as bdeg_cells_points does for the enumeration:
 * the start data of the polyhedral homotopies of Section 5, for k up to
 * BDEG_PIVOT_MAX_K.
 *   cell_masks [cap], normal_num [cap * k], normal_den [cap]: at most cap
 *   cells written (cap = 0: none; the arrays may then be NULL);
 *   *n_cells, *nvol, *tie: as for bdeg_pivot_points.
 * Cells come in no particular order; den sums to *nvol.
 */
int bdeg_pivot_cells(const int32_t *points, const int64_t *heights, int32_t N, int32_t k, uint64_t start_mask,
                     uint64_t cap, uint64_t *cell_masks, int64_t *normal_num, uint64_t *normal_den,
                     uint64_t *n_cells, bdeg_u128 *nvol, int32_t *tie);

/*
 * Consistency of x^A = b when rank A = r < m (Section 2, eq. "consistency"
 * and the global parametrization proposition): the system has solutions in
 * (C*)^n exactly when b^q = prod_i b_i^{q_i} = 1 for every q of a basis of
 * the integer left kernel {q in Z^m : q^T A = 0} (the columns of Q_0).  The
 * basis is saturated (it spans that whole lattice, not a sublattice), as the
 * test needs.  Host only; no device.
 *   A           m x n row-major int64 (as for bdeg_degree);
 *   b           m complex values as (re, im) double pairs, all nonzero;
 *   tol         *consistent = 1 when every |b^q - 1| <= tol;
 *   *residual   the largest |b^q - 1| (0 when r = m);
 *   *relations  m - r, the number of basis vectors q.
 * b^q is evaluated in double precision by repeated squaring of b_i^{|q_i|}.
 * Errors: BDEG_E_ARG (null pointer, bad sizes, a zero b_i), BDEG_E_OVERFLOW
 * (the host int64 algebra).
 */
int bdeg_consistency(const int64_t *A, int32_t m, int32_t n, const double *b, double tol,
                     int32_t *consistent, double *residual, int32_t *relations);

/*
 * Host prologue only (no device): rank, k, components and the point set
 * {0, v_1..v_n} the device would use (Euclid column elimination with a
 * pairwise-reduced saturated kernel basis).  points must hold (n+1)*n int32;
 * the first (n+1)*k are written, point 0 first.
 */
int bdeg_kernel_points(const int64_t *A, int32_t m, int32_t n, int32_t *k, int32_t *rank,
                       bdeg_u128 *components, int32_t *points);

/*
 * Serving: requests are admitted into device-resident slots as device memory
 * (budget bytes) allows, their work joins a shared device tile queue that is
 * drained in bounded steps, so requests overlap on the device; each result
 * is identical to the one bdeg_degree gives for the same input.
 *   bdeg_serve_open    start the engine (a host thread owns the device work).
 *   bdeg_serve_submit  copy A, queue the request, return a ticket (non-blocking).
 *   bdeg_serve_poll    BDEG_OK with *out filled (once), or BDEG_PENDING.
 *   bdeg_serve_wait    block until done, then as poll.
 *   bdeg_serve_latency time from submit to completion of a finished request,
 *                      in nanoseconds (BDEG_PENDING while it runs); valid
 *                      until bdeg_serve_close.
 *   bdeg_serve_close   finish queued work, stop the engine, free everything.
 * The budget bounds the device memory of admitted requests (a slot of about
 * 4.6 KiB each plus their share of the per-step work-unit buffer); requests
 * beyond it wait in arrival order.
 */
typedef struct bdeg_server bdeg_server;
int bdeg_serve_open(size_t device_mem_budget, bdeg_server **out);
int bdeg_serve_submit(bdeg_server *s, const int64_t *A, int32_t m, int32_t n, uint64_t seed,
                      int32_t lift_bits, uint64_t *ticket);
int bdeg_serve_poll(bdeg_server *s, uint64_t ticket, bdeg_result *out);
int bdeg_serve_wait(bdeg_server *s, uint64_t ticket, bdeg_result *out);
int bdeg_serve_latency(bdeg_server *s, uint64_t ticket, uint64_t *submit_to_done_ns);
int bdeg_serve_close(bdeg_server *s);

/*
 * Host only: the device work units for the candidates of N points in Z^k
 * with colex rank in [rank_lo, rank_hi), each at most max_cost candidates
 * where the subtree structure allows (0: the library's default for the
 * current device is not used; pass the cap explicitly).  Each unit is
 * reported as its colex rank interval [start, end): intervals[2u] = start,
 * intervals[2u+1] = end, in the order the device takes them.  *n_units is
 * always set; at most `cap` units are written (BDEG_E_NOMEM if more exist).
 */
int bdeg_plan_units(int32_t N, int32_t k, uint64_t rank_lo, uint64_t rank_hi, uint64_t max_cost,
                    uint64_t *intervals, size_t cap, size_t *n_units);

const char *bdeg_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* BDEG_H */
