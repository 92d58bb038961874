// Band key of one hash table (Algorithm 1: a table is keyed by the
// concatenation of K hash values).  The K values are folded with the
// SplitMix64 output function, seeded per table.
#pragma once
#include "common.hpp"

namespace ssh {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Fold of table l's K hash values of series s (hv values in h, stride 1)
__device__ __forceinline__ uint64_t band_fold(const uint64_t* h, int K, int l, uint64_t seed) {
  uint64_t k = mix64(seed + (uint64_t)(l + 1) * 0x9E3779B97F4A7C15ull);
  for (int t = 0; t < K; ++t) k = mix64(k ^ h[t]);
  return k == SSH_KEY_EMPTY ? SSH_KEY_EMPTY - 1 : k;
}

}  // namespace ssh
