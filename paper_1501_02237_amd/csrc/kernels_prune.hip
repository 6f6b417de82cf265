// Prefix pruning of the enumeration (paper Section 4.1: a set of points that
// is not a lower face cannot be extended to a lower facet).
//
// The candidates are split by their top d elements (colex): every d-subset F
// heads the subtree of candidates whose d largest points are F.  One
// wavefront per prefix F (lane j = point j):
//   * eliminates F's points fraction-free, exactly as the enumeration does
//     (lane j's residual after d - 1 steps: W = K + 1 - d spatial entries and a
//     height entry, all minors of the point matrix);
//   * decides whether F lies in a lower face.  Point j's height above the
//     hyperplanes through the lifted F is, up to a positive factor,
//     c_j + r_j . y with y in R^W free (r_j the spatial residual,
//     c_j = sign(prev) h_j).  By Farkas' lemma F lies in no lower face exactly
//     when some lambda >= 0 with sum lambda = 1 has sum lambda_j r_j = 0 and
//     sum lambda_j c_j < 0: the origin lies in the simplex of W + 1 residuals
//     r_A and the lifted simplex passes strictly below it.  Then no candidate
//     below F is a lower facet or a tie.  A float two-phase simplex over the
//     lanes (minimise sum lambda c under those equalities; lanes 0..W hold the
//     rows of the basis inverse) proposes the basis A, and the certificate is
//     checked exactly: W fraction-free Gauss-Jordan steps continue the
//     prefix's divisor chain (every entry stays a minor, inside the certified
//     widths), pivot on A minus one lane a0 and express
//     r_{a0} = sum mu_t r_{a_t}; it holds when every mu_t <= 0 (so lambda >= 0)
//     and a0 lies strictly below the hyperplane through F and the pivot lanes.
//     A wrong float answer can only miss a pruning, never cause one;
//   * emits, for a prefix that is kept, one enumeration unit per next element
//     c (the subtree of F + {c}), which the enumeration kernel then runs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"
#include "exact_div.hpp"
#include "wave_ratio.hpp"

namespace bdeg {
namespace dev {

constexpr int PK = BDEG_MAX_K; // widest point set
constexpr uint32_t PLOW31 = 0x7FFFFFFFu;

__device__ __forceinline__ int32_t prl32(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ uint64_t pbal(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t fkey(float f) { // order-preserving key of a float
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ double rl64f(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t r =
      ((uint64_t)(uint32_t)prl32((int32_t)(u >> 32), lane) << 32) | (uint32_t)prl32((int32_t)u, lane);
  return __longlong_as_double((long long)r);
}
__device__ __forceinline__ double bp64f(double v, int src) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int32_t)(u >> 32));
  const uint64_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int32_t)u);
  return __longlong_as_double((long long)((hi << 32) | lo));
}

// State of the float simplex (lanes 0..W hold the rows).
template <int W>
struct Lp {
  static constexpr int M = W + 1;
  double inv[W];  // row scales (uniform)
  double binv[M]; // lane i <= W: row i of the basis inverse
  double xb;      // lane i <= W: basic value of row i
  double pi[M];   // duals (uniform)
  int32_t mybasis; // lane i <= W: lane of row i's basic variable, -1 for an artificial
  uint64_t basic;  // basic lanes
};

// Lane j's column of the constraint matrix: (r_j / scale, 1).
template <int W>
__device__ __forceinline__ double col_entry(const Lp<W> &lp, const int32_t (&s)[W], int q) {
  return q < W ? (double)s[q] * lp.inv[q < W ? q : 0] : 1.0;
}

// One pivot: lane e enters, row lv leaves; col (lane i: row i of the entering
// column in the current basis), de = its reduced cost.
template <int W>
__device__ __forceinline__ void lp_pivot(Lp<W> &lp, int lv, int e, double col, double de) {
  constexpr int PM = W + 1;
  const int lane = (int)(threadIdx.x & 63);
  const double rp = 1.0 / rl64f(col, lv);
  double prow[PM];
#pragma unroll
  for (int q = 0; q < PM; q++) prow[q] = rl64f(lp.binv[q], lv) * rp;
  const double pxb = rl64f(lp.xb, lv) * rp;
#pragma unroll
  for (int q = 0; q < PM; q++) lp.binv[q] = lane == lv ? prow[q] : lp.binv[q] - col * prow[q];
  lp.xb = lane == lv ? pxb : lp.xb - col * pxb;
#pragma unroll
  for (int q = 0; q < PM; q++) lp.pi[q] += de * prow[q];
  const int old = prl32(lp.mybasis, lv);
  if (old >= 0) lp.basic &= ~(1ull << old);
  lp.basic |= 1ull << e;
  if (lane == lv) lp.mybasis = e;
}

// The entering column of lane e in the current basis, row i in lane i.
template <int W>
__device__ __forceinline__ double entering_col(const Lp<W> &lp, const int32_t (&s)[W], int e) {
  constexpr int PM = W + 1;
  double col = 0.0;
#pragma unroll
  for (int q = 0; q < PM; q++) {
    const double ae = q < W ? (double)prl32(s[q < W ? q : 0], e) * lp.inv[q < W ? q : 0] : 1.0;
    col += lp.binv[q] * ae;
  }
  return col;
}

// True when the prefix state (s, H1, H0, prev) with W columns lies in no lower
// face (certified).  lanes: the points outside the prefix.
template <int W>
__device__ __forceinline__ bool prefix_not_face(const int32_t (&s)[W], int32_t H1s, int32_t H0s, int32_t prevs,
                                                uint64_t lanes, uint32_t *pivots) {
  constexpr double TOL = 1e-9;
  constexpr uint32_t UMAX = 0xFFFFFFFFu;
  constexpr int M = W + 1, PW = W, PM = W + 1;
  constexpr int max_it = 4 * M + 12;
  const int lane = (int)(threadIdx.x & 63);
  const bool in = (lanes >> lane) & 1;
  Lp<W> lp;
  // scales: a_j = (r_j / max|r|, 1) per row, cost_j = sign(prev) h_j / max|h|
#pragma unroll
  for (int q = 0; q < PW; q++) {
    const float m = __uint_as_float(~wave_umin(~(in ? __float_as_uint(fabsf((float)s[q])) : 0u)));
    lp.inv[q] = m > 0.f ? 1.0 / (double)m : 1.0;
  }
  const double h = (double)H1s * 2147483648.0 + (double)(uint32_t)H0s;
  const float hm = __uint_as_float(~wave_umin(~(in ? __float_as_uint(fabsf((float)h)) : 0u)));
  const double cost = (prevs < 0 ? -h : h) * (hm > 0.f ? 1.0 / (double)hm : 1.0);
#pragma unroll
  for (int q = 0; q < PM; q++) {
    lp.binv[q] = lane == q ? 1.0 : 0.0;
    lp.pi[q] = q < M ? 1.0 : 0.0; // phase 1: every basic variable is an artificial of cost 1
  }
  lp.xb = lane == W ? 1.0 : 0.0;
  lp.mybasis = -1;
  lp.basic = 0;
  bool phase2 = false, stuck = false;
  int it = 0;
  for (;;) {
    // pricing: reduced cost of every non-basic lane (Dantzig's rule)
    double d = phase2 ? cost : 0.0;
#pragma unroll
    for (int q = 0; q < PM; q++)
      d -= lp.pi[q] * col_entry(lp, s, q);
    const bool cand = in && !((lp.basic >> lane) & 1) && d < -TOL;
    const uint32_t key = cand ? fkey((float)d) : UMAX;
    const uint32_t kmin = wave_umin(key);
    if (kmin == UMAX) {
      if (phase2) break;
      // end of phase 1: the artificials must be at zero (origin inside conv r)
      double art = 0.0;
      for (int i = 0; i < M; i++)
        if (prl32(lp.mybasis, i) < 0) art += rl64f(lp.xb, i);
      if (art > 1e-9) {
        stuck = true; // the origin is outside conv r: F lies in a lower face
        break;
      }
      // drive the zero-level artificials out (degenerate pivots)
      for (int i = 0; i < M && !stuck; i++) {
        if (prl32(lp.mybasis, i) >= 0) continue;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < PM; q++)
          v += rl64f(lp.binv[q], i) * col_entry(lp, s, q);
        const bool ok = in && !((lp.basic >> lane) & 1) && fabs(v) > TOL;
        const uint32_t mk = ok ? ~__float_as_uint(fabsf((float)v)) : UMAX;
        const uint32_t best = wave_umin(mk);
        if (best == UMAX) {
          stuck = true;
          continue;
        }
        const int e = __builtin_ctzll(pbal(mk == best));
        lp_pivot(lp, i, e, entering_col(lp, s, e), 0.0);
        it++;
      }
      if (stuck) break;
      // phase 2 duals: pi = c_B B^-1
      const double cbv = bp64f(cost, lane < M ? lp.mybasis : 0); // (every lane takes part)
      const double cb = lane < M ? cbv : 0.0;
#pragma unroll
      for (int q = 0; q < PM; q++) {
        const double v = cb * lp.binv[q];
        double sum = 0.0;
        for (int i = 0; i < M; i++) sum += rl64f(v, i);
        lp.pi[q] = sum;
      }
      phase2 = true;
      continue;
    }
    if (++it > max_it) break;
    const int e = __builtin_ctzll(pbal(key == kmin));
    const double de = rl64f(d, e);
    const double col = entering_col(lp, s, e);
    // ratio test over the rows; among equal ratios an artificial leaves first
    const bool rowc = lane < M && col > TOL;
    const uint32_t tk = rowc ? fkey((float)lp.xb * __builtin_amdgcn_rcpf((float)col)) : UMAX;
    const uint32_t tmin = wave_umin(tk);
    if (tmin == UMAX) break;
    const uint64_t tie = pbal(tk == tmin);
    const uint64_t art = tie & pbal(lp.mybasis < 0);
    lp_pivot(lp, __builtin_ctzll(art ? art : tie), e, col, de);
  }
  *pivots += (uint32_t)it;
  // the optimum sum lambda c is pi . b = pi[W] (b = e_W)
  const double piW = lp.pi[W];
  if (stuck || !phase2 || it > max_it || !(piW < -1e-12)) return false;
  // exact certificate; a0 = the basic lane with the largest weight
  int i0 = 0;
  double w0 = rl64f(lp.xb, 0);
  for (int i = 1; i < M; i++) {
    const double wi = rl64f(lp.xb, i);
    if (wi > w0) {
      w0 = wi;
      i0 = i;
    }
  }
  const int a0 = prl32(lp.mybasis, i0);
  if (a0 < 0 || ((lp.basic >> a0) & 1) == 0) return false;
  uint64_t piv = lp.basic & ~(1ull << a0);
  if (__builtin_popcountll(piv) != W) return false;
  int32_t x[PW];
#pragma unroll
  for (int q = 0; q < PW; q++) x[q] = s[q];
  int32_t H1 = H1s, H0 = H0s, prev = prevs;
#pragma unroll
  for (int t = 0; t < PW; t++) {
    if (t >= W) continue;
    const uint64_t c = pbal(x[t] != 0) & piv;
    if (!c) return false; // singular pivot set: no certificate
    const int pl = __builtin_ctzll(c);
    piv &= ~(1ull << pl);
    int32_t pc[PW];
#pragma unroll
    for (int r = 0; r < PW; r++) pc[r] = prl32(x[r], pl);
    const int32_t ph1 = prl32(H1, pl), ph0 = prl32(H0, pl);
    const int32_t p = pc[t];
    const Div dv = make_div(prev);
    const int32_t xt = x[t];
#pragma unroll
    for (int r = 0; r < PW; r++)
      if (r != t && r < W) x[r] = exdiv32((int64_t)p * x[r] - (int64_t)pc[r] * xt, dv);
    const int64_t A = (int64_t)p * H1 - (int64_t)ph1 * xt;
    const int64_t B = (int64_t)p * H0 - (int64_t)ph0 * xt;
    const int64_t hh = exdiv_split(A, B, dv);
    H1 = (int32_t)(hh >> 31);
    H0 = (int32_t)((uint32_t)hh & PLOW31);
    prev = p;
  }
  const bool dpos = prev > 0;
  bool ok = true;
#pragma unroll
  for (int t = 0; t < PW; t++) {
    if (t >= W) continue;
    const int32_t xa = prl32(x[t], a0);
    ok = ok && (dpos ? xa <= 0 : xa >= 0);
  }
  const int64_t sa = (int64_t)prl32(H1, a0) * ((int64_t)1 << 31) + (int64_t)(uint32_t)prl32(H0, a0);
  return ok && (dpos ? sa < 0 : sa > 0);
}

template <int W>
__global__ void __launch_bounds__(256) prune_kernel(PruneArgs a) {
  constexpr int PW = W;
  const int lane = (int)(threadIdx.x & 63);
  const bool valid = lane < a.N;
  const int K = a.K;
  const int d = K + 1 - W;   // prefix size
  const int lo_next = K - d; // the next element leaves room for K - d more below it
  uint32_t n_deg = 0, n_cut = 0, n_piv = 0;
  for (;;) {
    // every lane takes part in the claim (lane 0 adds one), read by index
    const uint32_t claim = atomicAdd(&a.cnt->next, lane == 0 ? 1u : 0u);
    const uint32_t item = (uint32_t)prl32((int32_t)claim, 0);
    if (item >= a.n_items) break;
    const uint64_t S = a.items[item];
    const int base = 63 - __builtin_clzll(S), e = __builtin_ctzll(S);
    int32_t x[PK];
#pragma unroll
    for (int r = 0; r < PK; r++) x[r] = (valid && r < K) ? a.pts[lane * K + r] - a.pts[base * K + r] : 0;
    int32_t H1 = 0, H0 = 0;
    if (valid) {
      const int64_t y = a.hts[lane] - a.hts[base];
      H1 = (int32_t)(y >> 31);
      H0 = (int32_t)((uint32_t)y & PLOW31);
    }
    // eliminate the prefix's other points, from the top down
    uint32_t used = 0;
    int32_t prev = 1;
    bool degen = false;
    uint64_t rest = S & ~(1ull << base);
    while (rest) {
      const int f = 63 - __builtin_clzll(rest);
      rest &= ~(1ull << f);
      int32_t pc[PK];
#pragma unroll
      for (int r = 0; r < PK; r++) pc[r] = prl32(x[r], f);
      int pr = -1;
#pragma unroll
      for (int r = 0; r < PK; r++)
        if (pr < 0 && r < K && !((used >> r) & 1) && pc[r] != 0) pr = r;
      if (pr < 0) { // the new point is affinely dependent on the others: no candidate below
        degen = true;
        break;
      }
      int32_t piv = 1, xp = 0;
#pragma unroll
      for (int r = 0; r < PK; r++)
        if (r == pr) {
          piv = pc[r];
          xp = x[r];
        }
      const int32_t ph1 = prl32(H1, f), ph0 = prl32(H0, f);
      const Div dv = make_div(prev);
#pragma unroll
      for (int r = 0; r < PK; r++)
        if (r < K && r != pr && !((used >> r) & 1)) x[r] = exdiv32((int64_t)piv * x[r] - (int64_t)pc[r] * xp, dv);
      const int64_t A = (int64_t)piv * H1 - (int64_t)ph1 * xp;
      const int64_t B = (int64_t)piv * H0 - (int64_t)ph0 * xp;
      const int64_t h = exdiv_split(A, B, dv);
      H1 = (int32_t)(h >> 31);
      H0 = (int32_t)((uint32_t)h & PLOW31);
      used |= 1u << pr;
      prev = piv;
    }
    if (degen) {
      n_deg++;
      continue;
    }
    // the W remaining rows, in increasing order
    int32_t s[PW];
#pragma unroll
    for (int q = 0; q < PW; q++) s[q] = 0;
    {
      int w = 0;
#pragma unroll
      for (int r = 0; r < PK; r++) {
        if (r < K && !((used >> r) & 1)) {
#pragma unroll
          for (int q = 0; q < PW; q++)
            if (q == w) s[q] = x[r];
          w++;
        }
      }
    }
    const uint64_t lanes = pbal(valid) & ~S;
    uint32_t its = 0;
    const bool cut = prefix_not_face<W>(s, H1, H0, prev, lanes, &its);
    n_piv += its;
    if (cut) {
      n_cut++;
      continue;
    }
    // units: lane c in [lo_next, e - 1] writes the runs of chunk c (mask F + c,
    // a run of the element after c) into bucket c
    if (lane >= lo_next && lane < e) {
      const int r0 = a.chunk_start[lane], r1 = a.chunk_start[lane + 1];
      uint32_t pos = a.bucket_off[lane] + atomicAdd(&a.bucket_cnt[lane], (uint32_t)(r1 - r0));
      for (int r = r0; r < r1; r++, pos++) {
        if (pos < a.cap_units) {
          Tile t;
          t.mask = W == 1 ? S : S | (1ull << lane); // (W = 1: the unit F, run [c, c])
          t.sys = 0;
          t.c_lo = a.run_lo[r];
          t.c_hi = a.run_hi[r];
          t.pad = 0;
          a.units[pos] = t;
        } else {
          atomicOr(&a.cnt->overflow, 1u);
        }
      }
    }
  }
  if (lane == 0) {
    if (n_deg) atomicAdd(&a.cnt->degenerate, n_deg);
    if (n_cut) atomicAdd(&a.cnt->pruned, n_cut);
    if (n_piv) atomicAdd(&a.cnt->pivots, (unsigned long long)n_piv);
  }
}

// Gather the buckets, largest next element (largest subtrees) first, into one
// list: thread i moves unit i of the bucketed array.
__global__ void __launch_bounds__(256) prune_compact_kernel(const Tile *in, Tile *out, const uint32_t *off,
                                                            const uint32_t *cnt, int c_lo, int c_hi, uint32_t cap) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= cap) return;
  uint32_t start = 0;
  for (int c = c_hi; c >= c_lo; c--) {
    if (i >= off[c] && i - off[c] < cnt[c]) {
      out[start + (i - off[c])] = in[i];
      return;
    }
    start += cnt[c];
  }
}

} // namespace dev

int launch_prune(void *stream, const PruneArgs &a) {
  if (a.W < 1 || a.W > PRUNE_WMAX || a.K < a.W || a.K > BDEG_MAX_K || a.N > 64) return BDEG_E_ARG;
  if (a.n_items == 0) return BDEG_OK;
  const void *f = nullptr;
  switch (a.W) {
    case 1: f = (const void *)dev::prune_kernel<1>; break;
    case 2: f = (const void *)dev::prune_kernel<2>; break;
    case 3: f = (const void *)dev::prune_kernel<3>; break;
    case 4: f = (const void *)dev::prune_kernel<4>; break;
    case 5: f = (const void *)dev::prune_kernel<5>; break;
    case 6: f = (const void *)dev::prune_kernel<6>; break;
    case 7: f = (const void *)dev::prune_kernel<7>; break;
    default: f = (const void *)dev::prune_kernel<8>; break;
  }
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0)
    return BDEG_E_DEVICE;
  uint64_t blocks = (uint64_t)per_cu * cus;
  const uint64_t need = ((uint64_t)a.n_items + 3) / 4;
  if (blocks > need) blocks = need;
  void *args[] = {(void *)&a};
  if (hipLaunchKernel(f, dim3((unsigned)blocks), dim3(256), args, 0, (hipStream_t)stream) != hipSuccess)
    return BDEG_E_DEVICE;
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

int launch_prune_compact(void *stream, const Tile *in, Tile *out, const uint32_t *off, const uint32_t *cnt, int c_lo,
                         int c_hi, uint32_t cap) {
  if (cap == 0) return BDEG_OK;
  if (c_lo < 0 || c_hi > 63 || c_lo > c_hi) return BDEG_E_ARG;
  hipLaunchKernelGGL(dev::prune_compact_kernel, dim3((cap + 255) / 256), dim3(256), 0, (hipStream_t)stream, in, out,
                     off, cnt, c_lo, c_hi, cap);
  return hipGetLastError() == hipSuccess ? BDEG_OK : BDEG_E_DEVICE;
}

} // namespace bdeg
