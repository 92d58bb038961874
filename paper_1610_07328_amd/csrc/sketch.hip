// Sliding-window sign sketch (Section 4.1 of Luo & Shrivastava, arXiv 1610.07328).
//
// bit i of a series = [ r . x[i*delta .. i*delta + W) >= 0 ].
//
// Fast path (W, delta) in {(80, 3), (64, 4), (128, 4), (30, 5)}: the windows
// of a work item (320 or 256 windows of one series) are matrix products on the
// matrix cores: with windows laid out in rows of 16, window 16 a + b is
// sum_k F[b][k] X[k][a], F[b][k] = r[k - delta b] (the filter on a band),
// X[k][a] = x[16 delta a + k], computed by 16x16x16 fp16 MFMAs (fp16 x fp16
// products exact in fp32, fp32 accumulation).  A second product gives each
// window's margin term: |F| with the sign-cleared staged samples (sum of
// |r^| |x^|, the L1 margin) or, for a filter with an fp16-subnormal entry, the
// 0/1 band with bf16(x^2) (the sum of squares).  The item's samples are staged
// once in LDS and loaded for the next item while one is computed.
// Any other (W, delta) takes the generic path: one window per lane with
// v_dot2_f32_f16 over fp16 sample pairs.
//
// Exactness: the reference bit is the sign of the float64 sum of the exact
// float32 products in ascending filter index.  The fast sum s16 differs
// from that float64 sum by at most c1a A + c0a with the L1 margin (see
// make_filter_args), else by at most
//     c1 ||r|| ||w|| + c2 sqrt(W) (||r|| + ||w||)
// (fp16 rounding of both operands, fp32 accumulation with up to W + 2
// roundings counted at 2^-23 each in any order, fp16 underflow/flush at 2^-14
// absolute, and the float64 sum's own rounding).  ||w|| is bounded from above
// with slack for the bf16 and fp32 roundings of the sum of squares (matrix
// path) or for the fp16 conversion (generic path).  A window with
// |s16| >= margin keeps the sign of s16; every other window (and every window
// of an item holding a sample with |x| >= 2^14 or a non-finite one) is queued
// and recomputed exactly like the reference, one window per lane, in float64.
// Queued windows are drained in rounds of 64 so a round keeps the whole wave
// busy (each lane loads its window's samples 16 at a time); a repaired 1 is
// OR-ed into the stored stream (the fast path stores 0 for every queued
// window).
#include <cmath>
#include <cstring>

#include "sketch_core.hpp"

namespace ssh {

__device__ __forceinline__ h2 as_h2(uint32_t u) { return __builtin_bit_cast(h2, u); }

__device__ __forceinline__ h2 pack_h2(float a, float b) {
  h2 v;
  v.x = (_Float16)a;
  v.y = (_Float16)b;
  return v;
}

__device__ __forceinline__ float fdot2(h2 a, h2 b, float c) {
  return __builtin_amdgcn_fdot2(a, b, c, false);
}

// Upper bound of the float64-vs-fast-path error for a window whose samples lie
// in a span with fp16 sum of squares E (fp32-accumulated).
__device__ __forceinline__ float window_margin(const FilterArgs& fa, float E, int span) {
  const float slack = 1.0f + 0x1p-20f;
  float wn = __builtin_sqrtf(E * (1.0f + 0x1p-9f) + (float)span * 0x1p-28f) * slack;
  float m = fa.c1 * fa.rnorm * wn + fa.c2 * fa.sqrtW * (fa.rnorm + wn);
  return m * slack;
}

// Stage samples [sbeg, sbeg + cap) of one series into LDS (zero past the end).
// Returns true on every lane when some staged sample is non-finite or has
// magnitude >= 2^14 (fp16 products could then overflow or lose the bound).
__device__ __forceinline__ bool stage_chunk(float* X, int cap, const float* __restrict__ x,
                                            int64_t base, int64_t m, int64_t sbeg) {
  bool bad = false;
  for (int e = lane_id(); e < cap; e += kWave) {
    int64_t g = sbeg + e;
    float v = g < m ? x[base + g] : 0.0f;
    bad |= !(__builtin_fabsf(v) < 16384.0f);
    X[e] = v;
  }
  return ballot64(bad) != 0;
}

// One repair round: up to 64 queued windows, one per lane, recomputed as the
// float64 sum of exact products in ascending filter index.
__device__ __forceinline__ void repair_round(const FilterArgs& fa, const float* __restrict__ x,
                             const int64_t* __restrict__ x_off, uint32_t* bits32,
                             const int64_t* __restrict__ bit_word_off, RepairQueue q,
                             unsigned long long& repaired) {
  const int lane = lane_id();
  int n = *q.count;
  int cnt = n < kWave ? n : kWave;
  int start = n - cnt;
  // This wave's earlier stores of stream words must be complete (in L2)
  // before the atomic ORs below reach the same words; the stores and the
  // atomics come from one wave, so a workgroup-scope fence (a wait on the
  // outstanding stores, no cache maintenance) orders them.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (lane < cnt) {
    uint32_t s = q.series[start + lane];
    uint32_t wi = q.window[start + lane];
    const float* xw = x + x_off[s] + (int64_t)wi * fa.delta;
    double acc = 0.0;
    // loads in groups of 16 (one wait per group), products in ascending order
    int k = 0;
#pragma clang loop unroll(disable)
    for (; k + 16 <= fa.W; k += 16) {
      float xv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = xw[k + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc = __builtin_fma((double)fa.r[k + u], (double)xv[u], acc);
    }
    for (; k < fa.W; ++k) acc = __builtin_fma((double)fa.r[k], (double)xw[k], acc);
    if (acc >= 0.0) {
      int64_t word = bit_word_off[s] + (wi >> 6);
      atomicOr(bits32 + 2 * word + ((wi >> 5) & 1), 1u << (wi & 31));
    }
  }
  if (lane == 0) *q.count = start;
  repaired += (unsigned long long)cnt;
  wave_sync_lds();
}

// The windows a wave recomputed, added to the global count once at its end
// (an atomic per repair round on one address serialises across the grid).
__device__ __forceinline__ void add_repaired(unsigned long long* repair_count,
                                             unsigned long long repaired) {
  if (lane_id() == 0 && repair_count && repaired) atomicAdd(repair_count, repaired);
}

template <int R>
__device__ __forceinline__ void push_flags(RepairQueue q, uint32_t flags, uint32_t s,
                                           uint32_t first_window) {
#pragma unroll
  for (int rho = 0; rho < R; ++rho) {
    if (flags & (1u << rho)) {
      int slot = atomicAdd(q.count, 1);
      q.series[slot] = s;
      q.window[slot] = first_window + rho;
    }
  }
}

// A work item is SUB = 16 ROWS windows of one series: ROWS rows of 16
// windows, computed 16 rows (one MFMA tile) at a time.
// Window 16 a + b (row a, column b) is the inner product of r with samples
// [D (16 a + b), + W), i.e. with samples k of row a's run [16 D a, + K) at
// k = D b + u (u < W).  So the item's sums are one matrix product
//     S[b][a] = sum_k F[b][k] X[k][a],  F[b][k] = r[k - D b] (0 off the band),
//                                       X[k][a] = x[16 D a + k],
// K = 16 ceil((15 D + W) / 16), done as K / 16 steps of the 16x16x16 fp16
// MFMA (products exact in fp32, fp32 accumulation).  The same product of the
// 0/1 band with bf16(x^2) gives every window's sum of squares, the norm the
// margin needs.  With F as the A operand, lane L ends up holding the four
// consecutive windows 16 (L % 16) + 4 (L / 16) + i, i = 0..3, of the tile.
// Whether the fast sum S of a window whose bf16 sum of squares (fp32-
// accumulated) is E has a trusted sign.  bf16 rounding of a square is below
// 2^-7 relative whatever the rounding direction, and the fp32 accumulation far
// below that, so ||w||^2 <= Q = E (1 + 2^-6) + W 2^-28 (the last term covers
// squares that underflow).  The error bound is alpha ||w|| + beta with
// alpha = c1 ||r|| + c2 sqrt(W) and beta = c2 sqrt(W) ||r||, so the sign is
// trusted when |S| - beta > 0 and (|S| - beta)^2 > alpha^2 Q.  In float32:
// y = |S| - b0 (b0 >= beta) and the test y > 0, y^2 > a2 Q.  Each of the
// five roundings (y, y^2, the fused Q, a2 Q, and a2 itself) is within 2^-24
// relative, and a2 carries a factor 1 + 2^-18 over alpha^2 that exceeds them
// all, so a pass implies |S| > alpha ||w|| + beta exactly.  No overflow:
// |S| < 2^35 and Q < 2^36 for the samples the fast path accepts (|x| < 2^14).
template <int W>
__device__ __forceinline__ bool mfma_sign_trusted(const FilterArgs& fa, float S, float E) {
  const float Q = __builtin_fmaf(E, 1.0f + 0x1p-6f, (float)W * 0x1p-28f);
  const float y = __builtin_fabsf(S) - fa.b0;
  return y > 0.0f && y * y > fa.a2 * Q;
}

// L1 = true: the margin comes from A = sum over the window of |r^_k| |x^_k|
// (fp16 values, an MFMA of the sign-cleared filter and samples), which needs
// no second staged copy of the samples; see make_filter_args for the bound.
// L1 = false (a filter with entries in fp16's subnormal range): the margin
// from the bf16 sum of squares E.
template <int W, int D, int ROWS, bool L1>
__global__ __launch_bounds__(256) void sketch_mfma_kernel(
    const float* __restrict__ x, const int64_t* __restrict__ x_off, int64_t N, FilterArgs fa,
    uint64_t* __restrict__ bits, const int64_t* __restrict__ bit_word_off,
    int32_t* __restrict__ nbits_out, unsigned long long* repair_count, int* err) {
  constexpr int SUB = 16 * ROWS;           // windows per item: ROWS rows of 16
  constexpr int TILES = (ROWS + 15) / 16;  // MFMA tiles of 16 rows
  constexpr int RS = 16 * D;               // samples between rows
  constexpr int KS = (15 * D + W + 15) / 16;  // k-steps
  constexpr int NS = (ROWS - 1) * RS + 16 * KS;  // samples an item reads
  constexpr int PF4 = (NS + 4 * kWave - 1) / (4 * kWave);  // rows of 256 samples
  constexpr int QCAP = SUB + kWave;
  static_assert(NS % 4 == 0 && RS % 4 == 0, "8-byte operand reads");
  static_assert(ROWS % 4 == 0, "whole stream words per item");

  // quad u of the item sits at slot u + u / 4 (one pad slot per four)
  __shared__ uint2 xh[kWavesPerBlock][PF4 * kWave * 5 / 4];  // fp16 quads of the samples
  __shared__ uint2 xq[kWavesPerBlock][L1 ? 1 : PF4 * kWave * 5 / 4];  // bf16 quads of squares
  __shared__ uint32_t qser[kWavesPerBlock][QCAP];
  __shared__ uint32_t qwin[kWavesPerBlock][QCAP];
  __shared__ uint16_t bw[kWavesPerBlock][ROWS];
  __shared__ int qn[kWavesPerBlock];

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int lane = lane_id();
  const int col = lane & 15, grp = lane >> 4;
  RepairQueue q{qser[w], qwin[w], &qn[w]};
  unsigned long long repaired = 0;  // windows this wave recomputed
  uint32_t* bits32 = reinterpret_cast<uint32_t*>(bits);
  if (lane == 0) qn[w] = 0;

  // A operands: F[b][k] and either |F| (L1) or the 0/1 band, b = lane % 16,
  // k = 16 t + 4 (lane / 16) + e
  half4 fr[KS];
  half4 fa1[KS];
  bf16x4 fo[KS];
#pragma unroll
  for (int t = 0; t < KS; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = 16 * t + 4 * grp + e - D * col;
      const bool in = u >= 0 && u < W;
      fr[t][e] = in ? (_Float16)fa.r[in ? u : 0] : (_Float16)0.0f;
      fa1[t][e] = __builtin_fabsf16(fr[t][e]);
      fo[t][e] = in ? (short)0x3F80 : (short)0;
    }
  }
  wave_sync_lds();

  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t s0 = (int64_t)blockIdx.x * kWavesPerBlock + w;
  ChunkItem cur;
  cur.s = N;
  if (s0 < N) {
    cur = series_item<W, D>(s0, x_off, bit_word_off, nbits_out, err);
    if (cur.nb == 0) cur = next_item<W, D, SUB>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
  }
  float pv[PF4][4];
  if (cur.s < N) load_item4<PF4>(x, cur, (int64_t)cur.c * SUB * D, pv);

  while (cur.s < N) {
    // stage the item's samples; flag it when one could overflow the fp16
    // products or is not finite
    bool bad = false;
#pragma unroll
    for (int i = 0; i < PF4; ++i) {
      const int p = lane + (lane >> 2) + kWave * 5 / 4 * i;  // slot of quad lane + 64 i
      xh[w][p] = make_uint2(pack_f16(pv[i][0], pv[i][1]), pack_f16(pv[i][2], pv[i][3]));
      if constexpr (!L1)
        xq[w][p] = make_uint2(pack_bf16(pv[i][0] * pv[i][0], pv[i][1] * pv[i][1]),
                              pack_bf16(pv[i][2] * pv[i][2], pv[i][3] * pv[i][3]));
#pragma unroll
      for (int e = 0; e < 4; ++e) bad |= !(__builtin_fabsf(pv[i][e]) < 16384.0f);
    }
    const bool unsafe = ballot64(bad) != 0;
    wave_sync_lds();

    // start loading the next item; it is consumed at the top of the next iteration
    const ChunkItem nxt = next_item<W, D, SUB>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
    if (nxt.s < N) load_item4<PF4>(x, nxt, (int64_t)nxt.c * SUB * D, pv);

    const int nb = cur.nb;
    const int c = cur.c;
    const uint2* xh2 = xh[w];
    const uint2* xq2 = xq[w];
#pragma unroll
    for (int tile = 0; tile < TILES; ++tile) {
      // B operands X[k][a], a = 16 tile + lane % 16, k = 16 t + 4 (lane / 16) + e:
      // four consecutive samples from sample 16 D a + 16 t + 4 (lane / 16); rows
      // past the item read its last row (their windows are not used)
      const int row = 16 * tile + col;
      const int rowc = row < ROWS ? row : ROWS - 1;
      float4v S = {0.0f, 0.0f, 0.0f, 0.0f}, E = {0.0f, 0.0f, 0.0f, 0.0f};
      const int b0 = (RS * rowc + 4 * grp) / 4;  // quad of the first sample
      const int b0s = b0 + (b0 >> 2);             // its slot; quad b0 + 4 t at b0s + 5 t
#pragma unroll
      for (int t = 0; t < KS; ++t) {
        const uint2 hv = xh2[b0s + 5 * t];
        S = __builtin_amdgcn_mfma_f32_16x16x16f16(fr[t], __builtin_bit_cast(half4, hv), S, 0, 0, 0);
        if constexpr (L1) {
          const uint2 av = make_uint2(hv.x & 0x7FFF7FFFu, hv.y & 0x7FFF7FFFu);  // |x^|
          E = __builtin_amdgcn_mfma_f32_16x16x16f16(fa1[t], __builtin_bit_cast(half4, av), E, 0, 0, 0);
        } else {
          const uint2 qv = xq2[b0s + 5 * t];
          E = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fo[t], __builtin_bit_cast(bf16x4, qv), E, 0,
                                                        0, 0);
        }
      }
      const int wl = 16 * row + 4 * grp;  // item-relative window of S[0]
      const int nvalid = row < ROWS ? nb - c * SUB - wl : 0;
      uint32_t nib = 0, flags = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nvalid) {
          const bool trusted = L1 ? __builtin_fabsf(S[i]) > __builtin_fmaf(fa.c1a, E[i], fa.c0a)
                                  : mfma_sign_trusted<W>(fa, S[i], E[i]);
          if (unsafe || !trusted) flags |= 1u << i;
          else if (S[i] >= 0.0f) nib |= 1u << i;
        }
      }
      // bits of windows 16 row .. + 15 from the four lanes sharing the row
      uint32_t v = nib << (4 * grp);
      v |= __shfl_xor(v, 16, kWave);
      v |= __shfl_xor(v, 32, kWave);
      if (grp == 0 && row < ROWS) bw[w][row] = (uint16_t)v;
      if (flags) push_flags<4>(q, flags, (uint32_t)cur.s, (uint32_t)(c * SUB + wl));
    }
    wave_sync_lds();
    const int nwords = (nb + 63) / 64;
    if (lane < ROWS / 2) {
      const int64_t wd = (int64_t)c * (ROWS / 4) + (lane >> 1);
      if (wd < nwords)
        bits32[2 * (cur.wo + wd) + (lane & 1)] = reinterpret_cast<const uint32_t*>(bw[w])[lane];
    }
    while (qn[w] >= kWave) repair_round(fa, x, x_off, bits32, bit_word_off, q, repaired);
    cur = nxt;
  }
  while (qn[w] > 0) repair_round(fa, x, x_off, bits32, bit_word_off, q, repaired);
  add_repaired(repair_count, repaired);
}

// ---------------------------------------------------------------------------
// generic path: any W <= SSH_MAX_W and delta, one window per lane
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sketch_generic_kernel(
    const float* __restrict__ x, const int64_t* __restrict__ x_off, int64_t N, FilterArgs fa,
    uint64_t* __restrict__ bits, const int64_t* __restrict__ bit_word_off,
    int32_t* __restrict__ nbits_out, unsigned long long* repair_count, int* err) {
  extern __shared__ unsigned char smem[];
  const int W = fa.W, D = fa.delta;
  const int XCAP = (kWave - 1) * D + W + 2;
  constexpr int QCAP = 2 * kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int lane = lane_id();
  // per wave: XCAP floats, 2*QCAP queue words, 2 stream words, 1 counter
  const size_t per_wave = (size_t)XCAP * 4 + 2 * QCAP * 4 + 2 * 4 + 4;
  unsigned char* mine = smem + per_wave * w;
  float* X = reinterpret_cast<float*>(mine);
  uint32_t* qs = reinterpret_cast<uint32_t*>(mine + (size_t)XCAP * 4);
  uint32_t* bw = qs + 2 * QCAP;
  int* qcount = reinterpret_cast<int*>(bw + 2);
  RepairQueue q{qs, qs + QCAP, qcount};
  unsigned long long repaired = 0;  // windows this wave recomputed
  uint32_t* bits32 = reinterpret_cast<uint32_t*>(bits);
  if (lane == 0) *qcount = 0;
  wave_sync_lds();
  const int PE = (W + 1) / 2;

  for (int64_t s = (int64_t)blockIdx.x * kWavesPerBlock + w; s < N;
       s += (int64_t)gridDim.x * kWavesPerBlock) {
    const int64_t base = x_off[s];
    const int64_t m = x_off[s + 1] - base;
    int nb = m >= W ? (int)((m - W) / D + 1) : 0;
    const int64_t wo = bit_word_off[s];
    if (bit_word_off[s + 1] - wo < (nb + 63) / 64) {
      if (lane == 0) atomicOr(err, 1);
      nb = 0;
    }
    if (lane == 0) nbits_out[s] = nb;
    const int nwords = (nb + 63) / 64;
    for (int c = 0; c * kWave < nb; ++c) {
      const bool unsafe = stage_chunk(X, XCAP, x, base, m, (int64_t)c * kWave * D);
      if (lane < 2) bw[lane] = 0;
      wave_sync_lds();
      const int wi = c * kWave + lane;
      if (wi < nb) {
        const float* P = X + lane * D;
        float acc = 0.0f, E = 0.0f;
        for (int p = 0; p < PE; ++p) {
          h2 v = pack_h2(P[2 * p], P[2 * p + 1]);
          acc = fdot2(v, as_h2(fa.even[p]), acc);
          E = fdot2(v, v, E);
        }
        const float M = window_margin(fa, E, 2 * PE);
        const bool flag = unsafe || !(__builtin_fabsf(acc) >= M);
        if (flag) {
          int slot = atomicAdd(qcount, 1);
          q.series[slot] = (uint32_t)s;
          q.window[slot] = (uint32_t)wi;
        } else if (acc >= 0.0f) {
          atomicOr(bw + (lane >> 5), 1u << (lane & 31));
        }
      }
      wave_sync_lds();
      if (lane < 2 && c < nwords) bits32[2 * (wo + c) + lane] = bw[lane];
      while (*qcount >= kWave) repair_round(fa, x, x_off, bits32, bit_word_off, q, repaired);
    }
  }
  while (*qcount > 0) repair_round(fa, x, x_off, bits32, bit_word_off, q, repaired);
  add_repaired(repair_count, repaired);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
uint16_t to_half_bits(float f) {
  _Float16 h = (_Float16)f;  // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}

float round_up_f32(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

// Absolute term c0a of the L1 margin for a filter of W taps whose margin
// weights (the |r^| of the derivation below) sum to l1r.
float l1_margin_abs(double l1r, int W) {
  const double u = 0x1p-11, e32 = 0x1p-23, k = W + 2;
  const double gam = k * e32 / (1.0 - k * e32);
  const double v = u / (1 - u);
  const double e64 = (W + 1) * 0x1p-53;
  return round_up_f32(0x1p-14 * (1 + v) * (1 + e64) * l1r / (1 - gam) * 1.01 * (1 + 0x1p-20));
}

ssh_status make_filter_args(const float* r, int W, int delta, FilterArgs& fa) {
  memset(&fa, 0, sizeof(fa));
  double n2 = 0.0;
  for (int k = 0; k < W; ++k) {
    if (!(__builtin_fabsf(r[k]) < 16384.0f)) return fail(SSH_EINVAL, "ssh_sketch: filter value not finite or |r| >= 2^14");
    fa.r[k] = r[k];
    n2 += (double)r[k] * (double)r[k];
  }
  auto rk = [&](int k) -> float { return (k >= 0 && k < W) ? r[k] : 0.0f; };
  for (int p = 0; p < SSH_MAX_W / 2 + 2; ++p) {
    fa.even[p] = (uint32_t)to_half_bits(rk(2 * p)) | ((uint32_t)to_half_bits(rk(2 * p + 1)) << 16);
  }
  const double u = 0x1p-11;               // fp16 unit roundoff (nearest)
  const double e32 = 0x1p-23;              // per-rounding fp32 error, counted generously
  const double k = W + 2;                  // roundings of the fp32 accumulation
  const double gam = k * e32 / (1.0 - k * e32);
  const double bound = (2 * u + u * u + gam * (1 + u) * (1 + u) + (W + 1) * 0x1p-53) * 1.01;
  fa.c1 = round_up_f32(bound > 1e-3 ? bound : 1e-3);
  fa.c2 = round_up_f32(0x1p-14 * (1 + u) * 1.01);
  fa.rnorm = round_up_f32(__builtin_sqrt(n2) * (1 + 0x1p-40));
  fa.sqrtW = round_up_f32(__builtin_sqrt((double)W));
  // L1 margin.  With r^ = fp16(r), x^ = fp16(x) and u = 2^-11: a filter entry
  // is 0 or has |r| >= 2^-14 (else l1 = 0), so |r - r^| <= v |r^| with
  // v = u / (1 - u); a sample has |x - x^| <= v |x^| or, below 2^-14 (flushed
  // or subnormal), |x - x^| <= 2^-14.  Then |r x - r^ x^| <= (2v + v^2) |r^ x^|
  // + 2^-14 (1 + v) |r^|.  The fast sum adds at most gam sum |r^ x^| of fp32
  // rounding (gam as above), the oracle's float64 sum differs from the exact
  // one by at most (W + 1) 2^-53 sum |r x|, and the MFMA's A is at least
  // (1 - gam) sum |r^ x^|.  So |s16 - s64| <= c1a A + c0a with the constants
  // below; the kernel trusts the sign when |s16| > fma(c1a, A, c0a), whose one
  // rounding the factor 1 + 2^-20 covers.
  {
    bool tiny = false;
    double l1r = 0.0;
    for (int k = 0; k < W; ++k) {
      const float a = __builtin_fabsf(r[k]);
      if (a != 0.0f && a < 0x1p-14f) tiny = true;
      l1r += __builtin_fabs((double)(_Float16)r[k]);
    }
    const double v = u / (1 - u);
    const double e64 = (W + 1) * 0x1p-53;
    const double rel = (2 * v + v * v + gam + e64 * (1 + v) * (1 + v)) / (1 - gam);
    fa.c1a = round_up_f32(rel * 1.01 * (1 + 0x1p-20));
    fa.c0a = l1_margin_abs(l1r, W);
    fa.l1 = tiny ? 0 : 1;
  }
  const double alpha = (double)fa.c1 * fa.rnorm + (double)fa.c2 * fa.sqrtW;
  fa.a2 = round_up_f32(alpha * alpha * (1 + 0x1p-18));
  fa.b0 = round_up_f32((double)fa.c2 * fa.sqrtW * fa.rnorm * (1 + 0x1p-20));
  fa.W = W;
  fa.delta = delta;
  return SSH_OK;
}

__device__ int g_sketch_err;

int take_sketch_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_sketch_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_sketch_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

// Device address of the flag word (shared with the multi-filter sketch).
int* sketch_err_ptr() {
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_sketch_err)) != hipSuccess) return nullptr;
  return err;
}

// Workgroups for the fast path: as many as the device holds at once (every
// wavefront then walks many series and its repair queue drains in full
// rounds, with no second, partly filled round of workgroups), and no more
// than the series need.
unsigned resident_grid(const void* kernel, int64_t N) {
  int dev = 0, cus = 0, per_cu = 0;
  unsigned cap = 2048;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) == hipSuccess &&
      cus > 0 && per_cu > 0)
    cap = (unsigned)(cus * per_cu);
  return grid_for(N, kWavesPerBlock, cap);
}

template <int WW, int DD, int RR>
static void launch_fast(const FilterArgs& fa, const float* x, const int64_t* x_off, int64_t N,
                        uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                        unsigned long long* rc, int* err, hipStream_t stream) {
  const dim3 blk(256);
  if (fa.l1) {
    const unsigned g = resident_grid(
        reinterpret_cast<const void*>(&sketch_mfma_kernel<WW, DD, RR, true>), N);
    sketch_mfma_kernel<WW, DD, RR, true><<<g, blk, 0, stream>>>(x, x_off, N, fa, bits,
                                                                 bit_word_off, nbits, rc, err);
  } else {
    const unsigned g = resident_grid(
        reinterpret_cast<const void*>(&sketch_mfma_kernel<WW, DD, RR, false>), N);
    sketch_mfma_kernel<WW, DD, RR, false><<<g, blk, 0, stream>>>(x, x_off, N, fa, bits,
                                                                  bit_word_off, nbits, rc, err);
  }
}

// Work-item sizes (rows of 16 windows) offered on the matrix-core path, and
// each shape's default: 20 rows hold the 315 windows of a 1024-sample series
// (W = 80, delta = 3) in one item.
bool sketch_tile_supported(int W, int delta, int rows) {
  const bool fast = (W == 80 && delta == 3) || (W == 64 && delta == 4) ||
                    (W == 128 && delta == 4) || (W == 30 && delta == 5);
  return fast && (rows == 8 || rows == 12 || rows == 16 || rows == 20);
}

static int default_rows(int W, int delta) { return W == 80 && delta == 3 ? 20 : 16; }

ssh_status sketch_launch(const float* x, const int64_t* x_off, int64_t N, const float* r, int W,
                         int delta, uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                         uint64_t* repair_count, hipStream_t stream, bool force_generic,
                         int tile_rows) {
  FilterArgs fa;
  ssh_status st = make_filter_args(r, W, delta, fa);
  if (st != SSH_OK) return st;
  if (N == 0) return SSH_OK;
  int* err = sketch_err_ptr();
  if (err == nullptr) return fail(SSH_EDEVICE, "ssh_sketch: cannot resolve error flag");
  unsigned long long* rc = reinterpret_cast<unsigned long long*>(repair_count);
  const unsigned grid = grid_for(N, kWavesPerBlock, 1 << 16);
  const dim3 blk(256);
  const int rows = tile_rows > 0 ? tile_rows : default_rows(W, delta);
#define SSH_FAST(WW, DD)                                                                       \
  if (!force_generic && W == WW && delta == DD) {                                              \
    switch (rows) {                                                                            \
      case 8: launch_fast<WW, DD, 8>(fa, x, x_off, N, bits, bit_word_off, nbits, rc, err, stream); break; \
      case 12: launch_fast<WW, DD, 12>(fa, x, x_off, N, bits, bit_word_off, nbits, rc, err, stream); break; \
      case 16: launch_fast<WW, DD, 16>(fa, x, x_off, N, bits, bit_word_off, nbits, rc, err, stream); break; \
      default: launch_fast<WW, DD, 20>(fa, x, x_off, N, bits, bit_word_off, nbits, rc, err, stream); break; \
    }                                                                                          \
    return check_launch("ssh_sketch");                                                         \
  }
  SSH_FAST(80, 3)
  SSH_FAST(64, 4)
  SSH_FAST(128, 4)
  SSH_FAST(30, 5)
#undef SSH_FAST
  const int XCAP = (kWave - 1) * delta + W + 2;
  const size_t per_wave = (size_t)XCAP * 4 + 2 * 2 * kWave * 4 + 2 * 4 + 4;
  const size_t shm = per_wave * kWavesPerBlock;
  if (shm > 160 * 1024) return fail(SSH_EUNSUPPORTED, "ssh_sketch: delta too large for LDS staging");
  sketch_generic_kernel<<<grid, blk, shm, stream>>>(x, x_off, N, fa, bits, bit_word_off, nbits,
                                                    rc, err);
  return check_launch("ssh_sketch");
}

}  // namespace ssh
