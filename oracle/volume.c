/*
 * Oracle: brute-force normalized volume by regular simplicial subdivision.
 *
 * TEST INFRASTRUCTURE ONLY.  Linked only by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; the product library never links or calls it.
 *
 * Plain C, exact, slow on purpose.  For a point set S = {a_0..a_{N-1}} in Z^k
 * with integer heights w_i (the lifting, Section 4), every (k+1)-subset
 * {c_0 < ... < c_k} is checked against the lower-facet system (eq.
 * ``lower-face``, strict form of eq. ``lower-d-face-again``):
 *
 *   rows x_j = (a_{c_j}, w_{c_j}) - (a_{c_0}, w_{c_0}),  j = 1..k   (k x (k+1))
 *   normal  n_i = (-1)^(k+i) det(x with column i removed),  i = 0..k
 *           (the cofactor vector: <x_j, n> = 0 for every row j)
 *   D = n_k = det of the spatial k x k block; |D| = normalized volume of the
 *           simplex (eq. ``simplex-vol``, read as |det(a_1-a_0, ..., a_k-a_0)|)
 *   D == 0      -> not a cell
 *   D < 0       -> negate n so that its last coordinate is positive (a lower
 *                  face has an inner normal with positive last coordinate)
 *   s_j = <(a_j, w_j) - (a_{c_0}, w_{c_0}), n>  for every other point j
 *   all s_j > 0 -> lower facet: add |D|
 *   no s_j < 0 but some s_j == 0 -> the lifting is not generic (a "tie")
 *
 * A lower facet's inner normal is (alpha, 1) with alpha_i = n_i / n_k (the
 * unique vector of eq. ``lower-d-face-again``): the linear functional
 * <., (alpha, 1)> is equal on the facet's lifted vertices and strictly larger
 * on every other lifted point.  oracle_cells_range lists the facets with the
 * numerators n_0..n_{k-1} and the denominator n_k = |D|.
 *
 * Determinants use Bareiss fraction-free elimination with row pivoting.
 * Every product, sum and difference is overflow-checked in __int128; an
 * overflow aborts the computation with ORACLE_E_OVERFLOW rather than return
 * a wrong value.  Subsets are visited in colex order, rank(c) = sum_i C(c_i, i+1);
 * a caller may restrict the visit to a rank range.  Worker threads take
 * contiguous rank chunks from a shared counter; each keeps its own partial sum.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_OVERFLOW (-2)
#define ORACLE_MAXK 20
#define ORACLE_MAXN 64

typedef __int128 i128;

uint64_t oracle_binom(int n, int r) {
  if (r < 0 || n < 0 || r > n) return 0;
  if (r > n - r) r = n - r;
  unsigned __int128 c = 1;
  for (int i = 1; i <= r; i++) {
    c = c * (unsigned)(n - r + i) / (unsigned)i;
    if (c > UINT64_MAX) return UINT64_MAX;
  }
  return (uint64_t)c;
}

typedef struct {
  const int64_t *pts;
  const int64_t *hts;
  int N, k;
  uint64_t lo, hi, chunk;
  uint64_t next; /* shared chunk counter (atomic) */
  int err;       /* shared error flag (atomic) */
  /* optional cell list: facets beyond cap are counted, not stored */
  uint64_t cap;
  uint64_t *masks;
  int64_t *num; /* cap x k */
  uint64_t *den;
  uint64_t n_emit; /* shared (atomic) */
} job_t;

typedef struct {
  job_t *job;
  i128 vol;
  uint64_t cells, dzero;
  int tie, err;
} worker_t;

static int mul_ck(i128 a, i128 b, i128 *r) { return __builtin_mul_overflow(a, b, r); }
static int sub_ck(i128 a, i128 b, i128 *r) { return __builtin_sub_overflow(a, b, r); }
static int add_ck(i128 a, i128 b, i128 *r) { return __builtin_add_overflow(a, b, r); }

/* determinant of the n x n matrix a (row stride ORACLE_MAXK); destroys a */
static int bareiss_det(i128 a[][ORACLE_MAXK], int n, i128 *det) {
  int sign = 1;
  i128 prev = 1;
  for (int t = 0; t < n - 1; t++) {
    int p = -1;
    for (int i = t; i < n; i++)
      if (a[i][t] != 0) { p = i; break; }
    if (p < 0) { *det = 0; return 0; }
    if (p != t) {
      for (int j = 0; j < n; j++) { i128 x = a[t][j]; a[t][j] = a[p][j]; a[p][j] = x; }
      sign = -sign;
    }
    for (int i = t + 1; i < n; i++)
      for (int j = t + 1; j < n; j++) {
        i128 u, v, w;
        if (mul_ck(a[t][t], a[i][j], &u) || mul_ck(a[i][t], a[t][j], &v) || sub_ck(u, v, &w)) return 1;
        a[i][j] = w / prev; /* exact (Sylvester's identity) */
      }
    prev = a[t][t];
  }
  *det = sign > 0 ? a[n - 1][n - 1] : -a[n - 1][n - 1];
  return 0;
}

/* colex unranking: c_0 < ... < c_k with rank = sum C(c_i, i+1) */
static void unrank(uint64_t rank, int N, int k, int *c) {
  for (int i = k; i >= 0; i--) {
    int v = i;
    while (v + 1 < N && oracle_binom(v + 1, i + 1) <= rank) v++;
    c[i] = v;
    rank -= oracle_binom(v, i + 1);
  }
}

/* colex successor; returns 0 when c was the last subset */
static int successor(int N, int k, int *c) {
  int i = 0;
  while (i <= k && c[i] + 1 == (i == k ? N : c[i + 1])) i++;
  if (i > k) return 0;
  c[i]++;
  for (int j = 0; j < i; j++) c[j] = j;
  return 1;
}

/* one candidate: returns 0 ok, 1 overflow; updates w */
static int test_candidate(const job_t *J, const int *c, worker_t *w) {
  const int k = J->k, N = J->N, d = k + 1;
  i128 x[ORACLE_MAXK][ORACLE_MAXK + 1];
  const int64_t *p0 = J->pts + (size_t)c[0] * k;
  for (int j = 1; j <= k; j++) {
    const int64_t *pj = J->pts + (size_t)c[j] * k;
    for (int q = 0; q < k; q++) x[j - 1][q] = (i128)pj[q] - p0[q];
    x[j - 1][k] = (i128)J->hts[c[j]] - J->hts[c[0]];
  }
  i128 nrm[ORACLE_MAXK + 1];
  /* D first (column k removed); the other cofactors only when D != 0 */
  for (int pass = 0; pass < 2; pass++) {
    for (int col = (pass == 0 ? k : 0); col < (pass == 0 ? k + 1 : k); col++) {
      i128 a[ORACLE_MAXK][ORACLE_MAXK];
      for (int r = 0; r < k; r++) {
        int cc = 0;
        for (int q = 0; q < d; q++)
          if (q != col) a[r][cc++] = x[r][q];
      }
      i128 det;
      if (bareiss_det(a, k, &det)) return 1;
      nrm[col] = ((k + col) % 2 == 0) ? det : -det;
    }
    if (pass == 0 && nrm[k] == 0) { w->dzero++; return 0; }
  }
  if (nrm[k] < 0)
    for (int q = 0; q < d; q++) nrm[q] = -nrm[q];
  int in[ORACLE_MAXN] = {0};
  for (int i = 0; i <= k; i++) in[c[i]] = 1;
  int zero = 0;
  for (int j = 0; j < N; j++) {
    if (in[j]) continue;
    const int64_t *pj = J->pts + (size_t)j * k;
    i128 s = 0;
    for (int q = 0; q < d; q++) {
      i128 y = q < k ? (i128)pj[q] - p0[q] : (i128)J->hts[j] - J->hts[c[0]];
      i128 t;
      if (mul_ck(y, nrm[q], &t) || add_ck(s, t, &s)) return 1;
    }
    if (s < 0) return 0; /* some point below the hyperplane: not a lower facet */
    if (s == 0) zero = 1;
  }
  if (zero) { w->tie = 1; return 0; }
  if (add_ck(w->vol, nrm[k], &w->vol)) return 1;
  w->cells++;
  if (J->masks) {
    for (int q = 0; q < d; q++)
      if (nrm[q] > INT64_MAX || nrm[q] < INT64_MIN) return 1;
    const uint64_t idx = __atomic_fetch_add((uint64_t *)&J->n_emit, 1, __ATOMIC_RELAXED);
    if (idx < J->cap) {
      uint64_t m = 0;
      for (int i = 0; i <= k; i++) m |= 1ull << c[i];
      J->masks[idx] = m;
      for (int q = 0; q < k; q++) J->num[idx * (uint64_t)k + q] = (int64_t)nrm[q];
      J->den[idx] = (uint64_t)nrm[k];
    }
  }
  return 0;
}

static void *worker_main(void *arg) {
  worker_t *w = (worker_t *)arg;
  job_t *J = w->job;
  int c[ORACLE_MAXK + 1];
  for (;;) {
    if (__atomic_load_n(&J->err, __ATOMIC_RELAXED)) break;
    uint64_t start = __atomic_fetch_add(&J->next, J->chunk, __ATOMIC_RELAXED);
    if (start >= J->hi) break;
    uint64_t end = start + J->chunk < J->hi ? start + J->chunk : J->hi;
    unrank(start, J->N, J->k, c);
    for (uint64_t r = start; r < end; r++) {
      if (test_candidate(J, c, w)) {
        w->err = 1;
        __atomic_store_n(&J->err, 1, __ATOMIC_RELAXED);
        return 0;
      }
      if (r + 1 < end) successor(J->N, J->k, c);
    }
  }
  return 0;
}

/*
 * Normalized-volume contribution of the candidates with colex rank in
 * [rank_lo, rank_hi) (pass rank_hi = UINT64_MAX for "all").
 *   pts: N x k row-major int64; hts: N int64 heights.
 *   out_vol: the sum of |D| over lower facets, as two 64-bit halves.
 *   out_tie: 1 if a non-generic lower face was seen.
 * Returns ORACLE_OK, ORACLE_E_ARG or ORACLE_E_OVERFLOW.
 */
static int run_range(job_t *JP, const int64_t *pts, const int64_t *hts, int N, int k, uint64_t rank_lo,
                     uint64_t rank_hi, int nthreads, uint64_t *out_vol_lo, uint64_t *out_vol_hi, int *out_tie,
                     uint64_t *out_cells, uint64_t *out_dzero) {
  if (!pts || !hts || k < 1 || k >= ORACLE_MAXK || N > ORACLE_MAXN || N < k + 1 || nthreads < 1)
    return ORACLE_E_ARG;
  uint64_t total = oracle_binom(N, k + 1);
  if (rank_hi > total) rank_hi = total;
  if (rank_lo > rank_hi) rank_lo = rank_hi;
  job_t J = *JP;
  J.pts = pts; J.hts = hts; J.N = N; J.k = k;
  J.lo = rank_lo; J.hi = rank_hi; J.next = rank_lo;
  uint64_t span = rank_hi - rank_lo;
  J.chunk = span / ((uint64_t)nthreads * 64) + 1;
  if (J.chunk > 65536) J.chunk = 65536;
  worker_t *ws = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!ws || !th) { free(ws); free(th); return ORACLE_E_ARG; }
  for (int i = 0; i < nthreads; i++) ws[i].job = &J;
  for (int i = 1; i < nthreads; i++) pthread_create(&th[i], 0, worker_main, &ws[i]);
  worker_main(&ws[0]);
  for (int i = 1; i < nthreads; i++) pthread_join(th[i], 0);
  i128 vol = 0;
  uint64_t cells = 0, dzero = 0;
  int tie = 0, err = 0;
  for (int i = 0; i < nthreads; i++) {
    if (ws[i].err || add_ck(vol, ws[i].vol, &vol)) err = 1;
    cells += ws[i].cells;
    dzero += ws[i].dzero;
    tie |= ws[i].tie;
  }
  free(ws);
  free(th);
  JP->n_emit = J.n_emit;
  if (err) return ORACLE_E_OVERFLOW;
  *out_vol_lo = (uint64_t)vol;
  *out_vol_hi = (uint64_t)(vol >> 64);
  *out_tie = tie;
  if (out_cells) *out_cells = cells;
  if (out_dzero) *out_dzero = dzero;
  return ORACLE_OK;
}

int oracle_nvol_range(const int64_t *pts, const int64_t *hts, int N, int k, uint64_t rank_lo,
                      uint64_t rank_hi, int nthreads, uint64_t *out_vol_lo, uint64_t *out_vol_hi,
                      int *out_tie, uint64_t *out_cells, uint64_t *out_dzero) {
  job_t J;
  memset(&J, 0, sizeof J);
  return run_range(&J, pts, hts, N, k, rank_lo, rank_hi, nthreads, out_vol_lo, out_vol_hi, out_tie, out_cells,
                   out_dzero);
}

/*
 * The lower facets among the candidates with colex rank in [rank_lo, rank_hi):
 * vertex masks (bit i = point i) and inner normals alpha = num / den (num:
 * k entries per facet, den = the facet's normalized volume |D| > 0), in no
 * particular order.  At most cap facets are stored; *out_count is the number
 * found (a count above cap asks for a larger buffer).  *out_tie as for the
 * volume.  A numerator outside int64 returns ORACLE_E_OVERFLOW.
 */
int oracle_cells_range(const int64_t *pts, const int64_t *hts, int N, int k, uint64_t rank_lo, uint64_t rank_hi,
                       int nthreads, uint64_t cap, uint64_t *masks, int64_t *num, uint64_t *den,
                       uint64_t *out_count, int *out_tie) {
  if (!masks || !num || !den || !out_count || !out_tie) return ORACLE_E_ARG;
  job_t J;
  memset(&J, 0, sizeof J);
  J.cap = cap;
  J.masks = masks;
  J.num = num;
  J.den = den;
  uint64_t lo, hi;
  int rc = run_range(&J, pts, hts, N, k, rank_lo, rank_hi, nthreads, &lo, &hi, out_tie, 0, 0);
  *out_count = J.n_emit;
  return rc;
}
