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
//   * One wavefront owns one subtree of candidates: the subsets whose top
//     elements are a fixed prefix (colex order), completed downward by a
//     depth-first walk.  Lane j holds lifted point j (N <= 64); when N <= 32
//     the point set is replicated in 2 (4, 8) lane groups so that that many
//     candidates are tested per step.
//   * Walking down fixes one more point c: its residual row is broadcast with
//     v_readlane (wave-uniform scalars) and every lane eliminates it from its
//     own residual by one fraction-free (Bareiss) step,
//         r'_i = (piv * r_i - rc_i * r_p) / prev,
//     dividing exactly by the previous pivot through its 2-adic inverse.  After
//     t steps a lane's residuals are the (t+1)x(t+1) minors of the chosen
//     difference rows bordered by its own point, so the work of the shared
//     prefix is done once for all candidates below it.  A chosen point whose
//     spatial residual vanishes makes every completion degenerate (D = 0):
//     the whole subtree is skipped.
//   * With k points fixed a lane's residual is (sigma_j, h_j): one spatial
//     column and the height column.  Adding candidate c gives
//         D = sigma_c   (the k x k spatial determinant, up to a sign shared by
//                        every value below),
//         s_j * prev = sigma_c * h_j - h_c * sigma_j  (the (k+1)-minor with
//                        row j: point j's height over the hyperplane, times D),
//     so the lower-facet test of a candidate is one 2x2 cross product per lane
//     and a wavefront ballot.
//   * Integer widths are certified on the host: spatial minors fit int32,
//     height minors int64, and products are formed in 128 bits.
//   * Sums of |D| are kept per wavefront and added to the system's 128-bit
//     accumulator with 64-bit atomics and an explicit carry.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdeg_internal.hpp"

namespace bdeg {
namespace dev {

constexpr int KMAX = BDEG_MAX_K;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- exact division
// divisor d = (-1)^neg * 2^e * odd; inv = odd^{-1} mod 2^64.
struct Div {
  uint64_t inv;
  uint32_t e;
  uint32_t neg;
};

__device__ __forceinline__ Div make_div(int32_t d) {
  Div r;
  uint32_t a = d < 0 ? (uint32_t)(-(int64_t)d) : (uint32_t)d;
  r.e = (uint32_t)__builtin_ctz(a);
  uint64_t odd = (uint64_t)(a >> r.e);
  uint64_t x = odd; // correct to 3 bits: odd * odd == 1 mod 8
  x *= 2 - odd * x; // 6
  x *= 2 - odd * x; // 12
  x *= 2 - odd * x; // 24
  x *= 2 - odd * x; // 48
  x *= 2 - odd * x; // 96
  r.inv = x;
  r.neg = d < 0;
  return r;
}

// x is an exact multiple of the divisor; only bits [e, e+32) of x are used.
__device__ __forceinline__ int32_t exdiv32(uint64_t x, const Div &d) {
  uint32_t q = (uint32_t)(x >> d.e) * (uint32_t)d.inv;
  return d.neg ? -(int32_t)q : (int32_t)q;
}
__device__ __forceinline__ int64_t exdiv64(u128 x, const Div &d) {
  uint64_t q = (uint64_t)(x >> d.e) * d.inv;
  return d.neg ? -(int64_t)q : (int64_t)q;
}

// ---------------------------------------------------------------- cross-lane helpers
__device__ __forceinline__ int32_t rl32(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int64_t rl64(int64_t v, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int32_t bp32(int32_t v, int src_lane) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
__device__ __forceinline__ int64_t bp64(int64_t v, int src_lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// ---------------------------------------------------------------- per-wave state
template <int W>
struct St {
  int32_t s[W > 0 ? W : 1]; // spatial residuals (W columns)
  int64_t h;                // height residual
  Div dv;                   // the pivot that produced this state
  int32_t prev;
};

struct Ctx {
  int npad_log2, G, g, j;
  uint64_t valid_lanes; // lanes holding a real point, all groups
  uint64_t rep_unit;    // bit 0 of every group
  uint64_t chosen_rep;  // chosen points, replicated in every group
  int L;                // forced prefix length
  int forced[KMAX + 1];
  uint64_t acc, cells;
  uint32_t tie;
  uint64_t nodes[KMAX];
  uint64_t pruned, leaves;
};

template <int K, int T>
struct Level {
  // st: residuals at depth T (T+1 points chosen, lowest `low`)
  static __device__ __forceinline__ void run(Ctx &cx, const St<K - T> &st, int low) {
    constexpr int W = K - T;
    int hi_c, lo_c;
    if (T + 1 < cx.L) {
      hi_c = lo_c = cx.forced[T + 1];
    } else {
      hi_c = low - 1;
      lo_c = K - T - 1;
    }
    if constexpr (T + 1 < K) {
      for (int c = hi_c; c >= lo_c; --c) {
        int32_t rc[W];
#pragma unroll
        for (int i = 0; i < W; i++) rc[i] = rl32(st.s[i], c);
        int p = -1;
#pragma unroll
        for (int i = 0; i < W; i++)
          if (p < 0 && rc[i] != 0) p = i;
        if (p < 0) { // chosen point affinely dependent on the prefix: D = 0 below
          cx.pruned++;
          continue;
        }
        const int64_t hc = rl64(st.h, c);
        int32_t piv = rc[0];
        int32_t rjp = st.s[0];
#pragma unroll
        for (int i = 1; i < W; i++)
          if (p == i) {
            piv = rc[i];
            rjp = st.s[i];
          }
        St<W - 1> ch;
#pragma unroll
        for (int i = 0; i < W - 1; i++) {
          const bool sh = i >= p;
          const int32_t src = sh ? st.s[i + 1] : st.s[i];
          const int32_t rcs = sh ? rc[i + 1] : rc[i];
          const uint64_t x = (uint64_t)((int64_t)piv * src) - (uint64_t)((int64_t)rcs * rjp);
          ch.s[i] = exdiv32(x, st.dv);
        }
        const u128 xh = (u128)((i128)piv * st.h) - (u128)((i128)hc * rjp);
        ch.h = exdiv64(xh, st.dv);
        ch.dv = make_div(piv);
        ch.prev = piv;
        const uint64_t saved = cx.chosen_rep;
        cx.chosen_rep |= cx.rep_unit << c;
        cx.nodes[T + 1]++;
        Level<K, T + 1>::run(cx, ch, c);
        cx.chosen_rep = saved;
      }
    } else {
      // leaf: k points chosen; candidates c add the last point
      const int npad = 1 << cx.npad_log2;
      const int G = cx.G;
      const uint64_t gmask = npad == 64 ? ~0ull : ((1ull << npad) - 1);
      const uint64_t prevflip = st.prev < 0 ? ~0ull : 0ull;
      const int32_t sj = st.s[0];
      const int64_t hj = st.h;
      for (int c0 = hi_c; c0 >= lo_c; c0 -= G) {
        const int cg = c0 - cx.g;
        const bool cvalid = cg >= lo_c;
        const int src = (cx.g << cx.npad_log2) + (cvalid ? cg : 0);
        int32_t sc;
        int64_t hc;
        if (G == 1) {
          sc = rl32(sj, c0);
          hc = rl64(hj, c0);
        } else {
          sc = bp32(sj, src);
          hc = bp64(hj, src);
        }
        const i128 t = (i128)sc * hj - (i128)hc * sj;
        const uint64_t m_lt = ballot(t < 0);
        const uint64_t m_nz = ballot(t != 0);
        const uint64_t m_scneg = ballot(sc < 0);
        const uint64_t m_scnz = ballot(sc != 0);
        uint64_t cand_bits = 0, gvalid = 0;
        for (int q = 0; q < G; q++) {
          const int cq = c0 - q;
          if (cq < lo_c) break;
          cand_bits |= 1ull << ((q << cx.npad_log2) + cq);
          gvalid |= gmask << (q << cx.npad_log2);
        }
        const uint64_t active = cx.valid_lanes & ~cx.chosen_rep & ~cand_bits & gvalid & m_scnz;
        const uint64_t flip = m_scneg ^ prevflip;
        const uint64_t neg = (m_lt ^ flip) & m_nz & active;
        const uint64_t zero = ~m_nz & active;
        for (int q = 0; q < G; q++) {
          const int cq = c0 - q;
          if (cq < lo_c) break;
          const uint64_t gm = gmask << (q << cx.npad_log2);
          if (!(m_scnz & gm)) continue; // D = 0
          cx.leaves++;
          if (neg & gm) continue;
          if (zero & gm) {
            cx.tie = 1;
            continue;
          }
          const int32_t sv = rl32(sj, cq);
          cx.acc += (uint64_t)(sv < 0 ? -(int64_t)sv : (int64_t)sv);
          cx.cells++;
        }
      }
    }
  }
};

template <int K>
__device__ __forceinline__ void process_tile(Ctx &cx, const SysDesc &sd, const int32_t *__restrict__ pts,
                                             const int64_t *__restrict__ hts, uint64_t mask) {
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
  cx.L = __builtin_popcountll(mask);
  uint64_t m = mask;
#pragma unroll
  for (int t = 0; t <= K; t++) {
    if (t < cx.L) {
      const int e = 63 - __builtin_clzll(m);
      cx.forced[t] = e;
      m ^= 1ull << e;
    } else {
      cx.forced[t] = 0;
    }
  }
  const int base = cx.forced[0];
  St<K> st;
#pragma unroll
  for (int i = 0; i < K; i++) st.s[i] = P[i] - rl32(P[i], base);
  st.h = w - rl64(w, base);
  st.dv.inv = 1;
  st.dv.e = 0;
  st.dv.neg = 0;
  st.prev = 1;
  cx.chosen_rep = cx.rep_unit << base;
  Level<K, 0>::run(cx, st, base);
}

template <int KLO, int KHI>
__global__ void __launch_bounds__(256) enum_kernel(const SysDesc *__restrict__ sys,
                                                   const int32_t *__restrict__ pts,
                                                   const int64_t *__restrict__ hts,
                                                   const Tile *__restrict__ tiles, uint32_t n_tiles,
                                                   SysAcc *__restrict__ acc, DevCounters *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  Ctx cx;
#pragma unroll
  for (int t = 0; t < KMAX; t++) cx.nodes[t] = 0;
  cx.pruned = cx.leaves = 0;
  uint64_t ntiles_done = 0;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&cnt->next_tile, 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= n_tiles) break;
    const Tile tl = tiles[t];
    const SysDesc sd = sys[tl.sys];
    cx.npad_log2 = sd.npad_log2;
    cx.G = 64 >> sd.npad_log2;
    cx.g = lane >> sd.npad_log2;
    cx.j = lane & ((1 << sd.npad_log2) - 1);
    uint64_t unit = 0, vl = 0;
    const uint64_t pm = sd.N >= 64 ? ~0ull : ((1ull << sd.N) - 1);
    for (int q = 0; q < cx.G; q++) {
      unit |= 1ull << (q << sd.npad_log2);
      vl |= pm << (q << sd.npad_log2);
    }
    cx.rep_unit = unit;
    cx.valid_lanes = vl;
    cx.acc = 0;
    cx.cells = 0;
    cx.tie = 0;
    switch (sd.k) {
#define BDEG_CASE(KK)                                      \
  case KK:                                                 \
    if constexpr (KK >= KLO && KK <= KHI)                  \
      process_tile<KK>(cx, sd, pts, hts, tl.mask);         \
    break;
      BDEG_CASE(1) BDEG_CASE(2) BDEG_CASE(3) BDEG_CASE(4) BDEG_CASE(5) BDEG_CASE(6)
      BDEG_CASE(7) BDEG_CASE(8) BDEG_CASE(9) BDEG_CASE(10) BDEG_CASE(11) BDEG_CASE(12)
#undef BDEG_CASE
      default:
        break;
    }
    ntiles_done++;
    if (lane == 0 && (cx.acc | cx.cells | cx.tie)) {
      SysAcc *a = &acc[tl.sys];
      const unsigned long long old = atomicAdd((unsigned long long *)&a->lo, (unsigned long long)cx.acc);
      if (old + cx.acc < old) atomicAdd((unsigned long long *)&a->hi, 1ull);
      atomicAdd((unsigned long long *)&a->cells, (unsigned long long)cx.cells);
      if (cx.tie) atomicOr(&a->tie, 1u);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 1; t < KHI; t++)
      if (cx.nodes[t]) atomicAdd((unsigned long long *)&cnt->nodes[t], (unsigned long long)cx.nodes[t]);
    atomicAdd((unsigned long long *)&cnt->pruned, (unsigned long long)cx.pruned);
    atomicAdd((unsigned long long *)&cnt->leaves, (unsigned long long)cx.leaves);
    atomicAdd((unsigned long long *)&cnt->tiles, (unsigned long long)ntiles_done);
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
    for (int t = 0; t < KMAX; t++) cnt->nodes[t] = 0;
    cnt->pruned = cnt->leaves = cnt->tiles = 0;
    cnt->next_tile = 0;
    cnt->pad = 0;
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

typedef void (*EnumFn)(const SysDesc *, const int32_t *, const int64_t *, const Tile *, uint32_t, SysAcc *,
                       DevCounters *);

static EnumFn enum_fn(int kmax) {
  switch (kmax) {
    case 1: return dev::enum_kernel<1, 1>;
    case 2: return dev::enum_kernel<1, 2>;
    case 3: return dev::enum_kernel<1, 3>;
    case 4: return dev::enum_kernel<1, 4>;
    case 5: return dev::enum_kernel<1, 5>;
    case 6: return dev::enum_kernel<1, 6>;
    case 7: return dev::enum_kernel<1, 7>;
    case 8: return dev::enum_kernel<1, 8>;
    case 9: return dev::enum_kernel<1, 9>;
    case 10: return dev::enum_kernel<1, 10>;
    case 11: return dev::enum_kernel<1, 11>;
    case 12: return dev::enum_kernel<1, 12>;
    default: return nullptr;
  }
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

int max_enum_blocks(int kmax, int waves_per_block) {
  EnumFn f = enum_fn(kmax);
  if (!f) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)f, waves_per_block * 64, 0) != hipSuccess)
    return 0;
  return per_cu * device_cu_count();
}

int launch_enumerate(void *stream, const SysDesc *d_sys, const int32_t *d_pts, const int64_t *d_heights,
                     const Tile *d_tiles, uint32_t n_tiles, SysAcc *d_acc, DevCounters *d_cnt, int kmax,
                     LaunchShape shape) {
  EnumFn f = enum_fn(kmax);
  if (!f) return BDEG_E_TOO_LARGE;
  if (n_tiles == 0) return BDEG_OK;
  int blocks = shape.blocks;
  const int wpb = shape.waves_per_block > 0 ? shape.waves_per_block : 4;
  if (blocks <= 0) blocks = max_enum_blocks(kmax, wpb);
  if (blocks <= 0) return BDEG_E_DEVICE;
  const uint64_t need = ((uint64_t)n_tiles + wpb - 1) / wpb;
  if ((uint64_t)blocks > need) blocks = (int)need;
  hipLaunchKernelGGL(f, dim3(blocks), dim3(wpb * 64), 0, (hipStream_t)stream, d_sys, d_pts, d_heights, d_tiles,
                     n_tiles, d_acc, d_cnt);
  return hip_ok(hipGetLastError());
}

} // namespace bdeg
