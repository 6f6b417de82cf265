// Exact division on the device: a divisor d = (-1)^neg * 2^e * odd is kept as
// e and inv = (-1)^neg * odd^{-1} mod 2^64, so that the quotient of an exact
// multiple x of d is ((x >> e) * inv) mod 2^w, for any width w that holds it.
// (Fraction-free elimination only ever divides exactly: Sylvester's identity.)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdeg {
namespace dev {

// divisor d = (-1)^neg * 2^e * odd; inv = (-1)^neg * odd^{-1} mod 2^64, so that
// an exact quotient is ((x >> e) * inv) mod 2^w.
struct Div {
  uint64_t inv;
  uint32_t e;
};

__device__ __forceinline__ Div make_div(int32_t d) {
  Div r;
  const uint32_t a = d < 0 ? (uint32_t)(-(int64_t)d) : (uint32_t)d;
  r.e = (uint32_t)__builtin_ctz(a);
  const uint32_t odd = a >> r.e;
  uint32_t x = odd; // odd * odd == 1 mod 8: 3 correct bits, doubled by each Newton step
  x *= 2u - odd * x;  // 6
  x *= 2u - odd * x;  // 12
  x *= 2u - odd * x;  // 24
  x *= 2u - odd * x;  // 48 -> 32 bits correct
  uint64_t y = x;
  y *= 2ull - (uint64_t)odd * y; // 64 bits correct
  r.inv = d < 0 ? (uint64_t)0 - y : y;
  return r;
}

// x is an exact multiple of the divisor and the quotient fits int32.
__device__ __forceinline__ int32_t exdiv32(int64_t x, const Div &d) {
  return (int32_t)((uint32_t)((uint64_t)x >> d.e) * (uint32_t)d.inv);
}
// (A * 2^31 + B) / d for an exact multiple whose quotient fits int64; e <= 30.
__device__ __forceinline__ int64_t exdiv_split(int64_t A, int64_t B, const Div &d) {
  const uint64_t y = ((uint64_t)A << (31 - d.e)) + (uint64_t)(B >> d.e);
  return (int64_t)(y * d.inv);
}

// (x / d) for an exact multiple x of d whose quotient fits int64.
__device__ __forceinline__ int64_t exdiv128(__int128 x, const Div &d) {
  return (int64_t)((uint64_t)(x >> d.e) * d.inv);
}

} // namespace dev
} // namespace bdeg
