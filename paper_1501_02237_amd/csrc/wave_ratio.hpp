// Exact wave-wide minimum of ratios num / den (num signed, den > 0), used by
// the cell walk's pivot (and the DPP minimum by the prefix filter's pricing).
//
// The ratios are screened in float first: each lane converts |num| and den
// without cancellation (both halves of |num| are non-negative), takes the
// reciprocal and the product, and maps the float onto an unsigned key whose
// order is the float order (sign bit set for non-negative values, all bits
// inverted for negative ones).  Every rounding step is within one ulp, so the
// float is within a relative 2^-21 of the exact ratio and keeps its sign; a
// DPP minimum over the keys then bounds the exact minimum.  Every lane whose
// exact ratio is the minimum has a key within 64 ulps (a factor of at least
// 1 + 2^-17) of the smallest key, so only those lanes can win; when there are
// several they are compared exactly, with 128-bit cross products, one by one.
// Nonzero ratios are at least 2^-31 in magnitude (|num| >= 1, den < 2^31), far
// from the float subnormals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdeg {
namespace dev {

// Wave-wide minimum of an unsigned key (every lane active): a row-wise shift
// scan with DPP, then the row broadcasts; lane 63 ends with the minimum.
__device__ __forceinline__ uint32_t wave_umin(uint32_t v) {
  constexpr int UMAX = -1; // identity of the minimum for lanes without a source
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x111, 0xf, 0xf, false)); // row_shr:1
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x112, 0xf, 0xf, false)); // row_shr:2
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x114, 0xf, 0xf, false)); // row_shr:4
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x118, 0xf, 0xf, false)); // row_shr:8
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x142, 0xa, 0xf, false)); // row_bcast:15
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(UMAX, (int)v, 0x143, 0xc, 0xf, false)); // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Order-preserving unsigned key of num / den (den > 0) in float.
__device__ __forceinline__ uint32_t ratio_key(int64_t num, int32_t den) {
  const uint64_t mag = num < 0 ? (uint64_t)0 - (uint64_t)num : (uint64_t)num;
  const float fm = __builtin_fmaf((float)(uint32_t)(mag >> 32), 4294967296.0f, (float)(uint32_t)mag);
  const float r = (num < 0 ? -fm : fm) * __builtin_amdgcn_rcpf((float)den);
  const uint32_t u = __float_as_uint(r);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct RatioMin {
  int lane;       // lowest lane with the minimal ratio, -1 when no lane has a candidate
  uint64_t lanes; // every lane with the minimal ratio
};

// Exact minimum of num / den over the lanes with den > 0 (den <= 0: no
// candidate).  Every lane must be active.
// The minimum over the lanes with a candidate (has), given each lane's key.
__device__ __forceinline__ RatioMin ratio_min_keyed(uint32_t key, bool has, int64_t num, int32_t den) {
  constexpr uint32_t BAND = 64;
  const uint32_t kmin = wave_umin(key);
  RatioMin r;
  r.lane = -1;
  r.lanes = 0;
  if (kmin == 0xFFFFFFFFu) return r;
  uint64_t near = __builtin_amdgcn_ballot_w64(has && key - kmin <= BAND);
  r.lane = __builtin_ctzll(near);
  r.lanes = 1ull << r.lane;
  near &= near - 1;
  if (!near) return r;
  // several lanes in the band: exact comparison, one by one
  const int32_t nlo = (int32_t)(uint32_t)num, nhi = (int32_t)((uint64_t)num >> 32);
  auto num_of = [&](int j) {
    return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(nhi, j) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(nlo, j));
  };
  int64_t bn = num_of(r.lane);
  int32_t bd = __builtin_amdgcn_readlane(den, r.lane);
  while (near) {
    const int j = __builtin_ctzll(near);
    near &= near - 1;
    const int64_t jn = num_of(j);
    const int32_t jd = __builtin_amdgcn_readlane(den, j);
    const __int128 lhs = (__int128)jn * bd, rhs = (__int128)bn * jd;
    if (lhs < rhs) {
      r.lane = j;
      r.lanes = 1ull << j;
      bn = jn;
      bd = jd;
    } else if (lhs == rhs) {
      r.lanes |= 1ull << j;
    }
  }
  return r;
}

__device__ __forceinline__ RatioMin ratio_min(int64_t num, int32_t den) {
  const bool has = den > 0;
  return ratio_min_keyed(has ? ratio_key(num, has ? den : 1) : 0xFFFFFFFFu, has, num, den);
}

// float |num| as ratio_key rounds it, for a numerator shared by many minima
__device__ __forceinline__ float ratio_num(uint64_t mag) {
  return __builtin_fmaf((float)(uint32_t)(mag >> 32), 4294967296.0f, (float)(uint32_t)mag);
}

// ratio_min for num >= 0 with fnum = ratio_num(num) computed once by the
// caller: the same keys, bit for bit (a ratio >= 0 has its sign bit clear).
__device__ __forceinline__ RatioMin ratio_min_nonneg(float fnum, int64_t num, int32_t den) {
  const bool has = den > 0;
  const float r = fnum * __builtin_amdgcn_rcpf((float)(has ? den : 1));
  return ratio_min_keyed(has ? (__float_as_uint(r) | 0x80000000u) : 0xFFFFFFFFu, has, num, den);
}

} // namespace dev
} // namespace bdeg
