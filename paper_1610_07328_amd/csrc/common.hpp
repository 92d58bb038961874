// Internal helpers shared by the HIP sources of the SSH library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ssh.h"

namespace ssh {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// host-side error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
ssh_status fail(ssh_status code, const std::string& msg);
ssh_status check_launch(const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Number of workgroups for a grid-stride launch over `items` work units with
// `per_block` units handled per workgroup per round.
inline unsigned grid_for(int64_t items, int64_t per_block, int64_t cap = 65536) {
  int64_t g = ceil_div(items, per_block);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Top bits of a band key that the hash tables are sorted on (and that the
// probe searches): 24 while N <= 2^24, where a bucket's run holds on average
// at most one entry of another key (the probe compares full keys), else 32.
// Three radix passes instead of four.
__host__ __device__ inline int table_sort_bits(int64_t N) {
  return N <= ((int64_t)1 << 24) ? 24 : 32;
}

// ---------------------------------------------------------------------------
// device-side helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Linear workgroup index renumbered so that each XCD owns a contiguous range.
// Workgroups are dispatched to the 8 XCDs in turn by linear id g (XCD g mod
// 8); this returns the bijection of [0, G) that gives XCD x the indexes
// x per + min(x, rem) .. + per (+1 for x < rem), per = G / 8, rem = G mod 8.
// Work that consecutive indexes write side by side then meets in one L2.
__device__ __forceinline__ int64_t xcd_linear_block() {
  const int64_t G = (int64_t)gridDim.x * gridDim.y;
  const int64_t g = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
  const int64_t xcd = g & 7, per = G >> 3, rem = G & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + (g >> 3);
}

// all lanes of the wave see each other's LDS writes issued before this point
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_bcast(T v, int src) {
  return __shfl(v, src, kWave);
}

// inclusive prefix sum over the wave (lane order)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t t = __shfl_up(v, d, kWave);
    if (l >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

}  // namespace ssh
