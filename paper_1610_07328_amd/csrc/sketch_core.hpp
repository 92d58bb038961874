// Pieces shared by the sign-sketch kernels (Section 4.1): the filter's
// margin constants, the work items a resident grid walks, and staging loads.
#pragma once

#include "common.hpp"

namespace ssh {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

struct FilterArgs {
  float r[SSH_MAX_W];                // float32 filter, float64 repair path
  uint32_t even[SSH_MAX_W / 2 + 2];  // fp16 pairs (r[2p], r[2p+1]), r[W] = 0
  float c1;                          // relative margin factor
  float c2;                          // underflow margin factor
  float rnorm;                       // ||r||_2, rounded up
  float sqrtW;                       // sqrt(W), rounded up
  float a2;                          // (c1 rnorm + c2 sqrtW)^2 (1 + 2^-18), rounded up
  float b0;                          // c2 sqrtW rnorm (1 + 2^-20), rounded up
  float c1a;                         // relative factor of the L1 margin (no tiny r)
  float c0a;                         // absolute term of the L1 margin
  int32_t l1;                        // no r with 0 < |r| < 2^-14: the L1 margin applies
  int32_t W;
  int32_t delta;
};

struct RepairQueue {
  uint32_t* series;
  uint32_t* window;
  int* count;
};

constexpr int kWavesPerBlock = 4;

// ---------------------------------------------------------------------------
// work items of the fast path: chunks of SUB consecutive windows of a series,
// walked by a wave striding over series
// ---------------------------------------------------------------------------
struct ChunkItem {
  int64_t s;     // series (>= N: no item)
  int c;         // chunk of the series
  int nb;        // bits of the series
  int64_t base;  // first sample
  int64_t m;     // samples of the series
  int64_t wo;    // first stream word
};

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Header of series s (nb = 0 when the stream capacity is too small), and the
// series' bit count recorded.  Everything here is wave-uniform: every lane
// stores the same value (no lane-dependent branch, so the header stays in
// scalar registers).
template <int W, int D>
__device__ __forceinline__ ChunkItem series_item(int64_t s, const int64_t* __restrict__ x_off,
                                                 const int64_t* __restrict__ bit_word_off,
                                                 int32_t* __restrict__ nbits_out, int* err) {
  ChunkItem it;
  it.s = uniform64(s);
  it.c = 0;
  it.base = uniform64(x_off[it.s]);
  it.m = uniform64(x_off[it.s + 1]) - it.base;
  int nb = it.m >= W ? (int)((it.m - W) / D + 1) : 0;
  it.wo = uniform64(bit_word_off[it.s]);
  if (uniform64(bit_word_off[it.s + 1]) - it.wo < (nb + 63) / 64) {
    atomicOr(err, 1);
    nb = 0;
  }
  nbits_out[it.s] = nb;
  it.nb = nb;
  return it;
}

// The item after `it` for a wave striding over series by `stride`: the next
// chunk of the same series, else the first chunk of the next series that has
// at least one bit.
template <int W, int D, int SUB>
__device__ __forceinline__ ChunkItem next_item(ChunkItem it, int64_t N, int64_t stride,
                                               const int64_t* __restrict__ x_off,
                                               const int64_t* __restrict__ bit_word_off,
                                               int32_t* __restrict__ nbits_out, int* err) {
  if ((it.c + 1) * SUB < it.nb) {
    ++it.c;
    return it;
  }
  for (int64_t s = it.s + stride; s < N; s += stride) {
    ChunkItem n = series_item<W, D>(s, x_off, bit_word_off, nbits_out, err);
    if (n.nb > 0) return n;
  }
  it.s = N;
  return it;
}

// ---------------------------------------------------------------------------
// fast path on the matrix cores
// ---------------------------------------------------------------------------
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}

__device__ __forceinline__ uint32_t pack_f16(float a, float b) {
  const f32x2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2v));
}

// Samples 4p .. 4p + 3 (p = lane + 64 i) of an item starting at sample sb, one
// 16-byte load each, through a buffer resource whose range ends at the
// series' last sample (or past what the item needs): samples past the series
// read as zero (each dword is range-checked on its own).
template <int PF4>
__device__ __forceinline__ void load_item4(const float* __restrict__ x, const ChunkItem& it,
                                           int64_t sb, float (&pv)[PF4][4]) {
  const int lane = lane_id();
  const int64_t rem = it.m - sb;  // > 0 for an item
  const int64_t need = 4 * kWave * PF4;
  const int nrec = (int)((rem < need ? rem : need) * 4);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(x + it.base + sb), 0, nrec, 0x00020000);
#pragma unroll
  for (int i = 0; i < PF4; ++i) {
    // the builtin's own vector type, indexed directly
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * lane, 4 * kWave * i * 4, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) pv[i][e] = __builtin_bit_cast(float, (uint32_t)v[e]);
  }
}

// Host side (sketch.hip): filter checks and margin constants, fp16 bits and
// upward rounding to float, the resident grid size of a kernel, the device
// address of the sketch kernels' error flag word, and the L1 margin's
// absolute term for given margin weights.
ssh_status make_filter_args(const float* r, int W, int delta, FilterArgs& fa);
uint16_t to_half_bits(float f);
float round_up_f32(double v);
unsigned resident_grid(const void* kernel, int64_t N);
int* sketch_err_ptr();
float l1_margin_abs(double l1r, int W);

}  // namespace ssh
