// The seeded lifting (Section 4: heights w(a) of a generic lifting), shared by
// the host and the device so that a redraw made inside a captured device pass
// gives exactly the heights a host-driven redraw would.
//
// Key of (seed, system, attempt): SplitMix64's finaliser (Steele, Lea, Flood
// 2014) applied twice to the seed mixed with the system and attempt numbers
// and a library tag.  Height of point j: the top `bits` bits of the finaliser
// of key + (j + 1) * golden-ratio increment (a counter-based stream).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdeg {

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t lift_key(uint64_t seed, uint32_t sys_index, uint32_t attempt) {
  const uint64_t LIB_TAG = 0xB0E6D0C5B0E6D0C5ull;
  const uint64_t z = seed ^ LIB_TAG ^ ((uint64_t)(sys_index + 1) * 0x9E3779B97F4A7C15ull) ^
                     ((uint64_t)(attempt + 1) * 0xD1B54A32D192ED03ull);
  return mix64(mix64(z));
}

// height of point j in [0, 2^bits), 1 <= bits <= 63
__host__ __device__ inline int64_t lift_height(uint64_t key, int j, int bits) {
  return (int64_t)(mix64(key + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

} // namespace bdeg
