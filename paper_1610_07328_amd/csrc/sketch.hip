// Sliding-window sign sketch (Section 4.1 of Luo & Shrivastava, arXiv 1610.07328).
//
// bit i of a series = [ r . x[i*delta .. i*delta + W) >= 0 ].
//
// Fast path: one wavefront per series chunk; each lane owns R consecutive
// windows and keeps the union of their samples in registers as packed fp16
// pairs, so every loaded sample feeds several windows.  Products are fp16 x
// fp16 (exact in fp32) accumulated in fp32 by v_dot2_f32_f16.  The fp16
// filter pairs sit in LDS and are read at their point of use.  The grid is capped at 2048 workgroups, so each wavefront walks
// many series and its repair queue drains in full rounds.
//
// Exactness: the reference bit is the sign of the float64 sum of the exact
// float32 products in ascending filter index.  The fast-path sum s16 differs
// from that float64 sum by at most
//     c1 ||r|| ||w|| + c2 sqrt(W) (||r|| + ||w||)
// (fp16 rounding of both operands, fp32 accumulation with up to W + 2
// roundings counted at 2^-23 each, fp16 underflow/flush at 2^-14 absolute,
// and the float64 sum's own rounding).  ||w|| is bounded from above by the
// norm of the lane's whole sample span, computed from the same fp16 values
// with the conversion and accumulation slack added.  A window with
// |s16| >= margin keeps the sign of s16; every other window (and every window
// of a chunk holding a sample with |x| >= 2^14 or a non-finite one) is queued
// and recomputed exactly like the reference, one window per lane, in float64.
// Queued windows are drained in rounds of 64 so a round keeps the whole wave
// busy (each lane loads its window's samples 16 at a time); a repaired 1 is
// OR-ed into the stored stream (the fast path stores 0 for every queued
// window).
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace ssh {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

struct FilterArgs {
  float r[SSH_MAX_W];                // float32 filter, float64 repair path
  uint32_t even[SSH_MAX_W / 2 + 2];  // fp16 pairs (r[2p], r[2p+1]), r[W] = 0
  uint32_t odd[SSH_MAX_W / 2 + 2];   // fp16 pairs (r[2p-1], r[2p]), r[-1] = r[W] = 0
  float c1;                          // relative margin factor
  float c2;                          // underflow margin factor
  float rnorm;                       // ||r||_2, rounded up
  float sqrtW;                       // sqrt(W), rounded up
  int32_t W;
  int32_t delta;
};

struct RepairQueue {
  uint32_t* series;
  uint32_t* window;
  int* count;
};

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
                             unsigned long long* repair_count) {
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
  if (lane == 0) {
    *q.count = start;
    if (repair_count) atomicAdd(repair_count, (unsigned long long)cnt);
  }
  wave_sync_lds();
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

// lane's R bits at chunk-relative window position wl into the LDS words bw
template <int R>
__device__ __forceinline__ void or_bits(uint32_t* bw, int wl, uint32_t b) {
  if (!b) return;
  int word = wl >> 5, sh = wl & 31;
  atomicOr(bw + word, b << sh);
  if (sh + R > 32) atomicOr(bw + word + 1, b >> (32 - sh));
}

constexpr int kWavesPerBlock = 4;

// ---------------------------------------------------------------------------
// fast path: compile-time W, delta and R windows per lane
// ---------------------------------------------------------------------------
// A work item is one chunk of SUB = 64 R windows of one series.  The chunk's
// samples are staged in LDS as fp16 pairs, converted once: ev[p] holds
// (x[2p], x[2p+1]) and od[p] holds (x[2p-1], x[2p]) (chunk-relative indices),
// so a lane whose span starts at an even sample reads ev and one starting at
// an odd sample reads od.  While a chunk is computed, the samples of the
// wave's next chunk are already being loaded into registers.
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

// Samples 2p and 2p+1 (p = lane + 64 i) of a chunk starting at sample sb,
// read through a buffer resource whose range ends at the series' last sample
// (or past what the chunk needs), so samples past the series read as zero
// without any per-load bounds arithmetic.
template <int PF>
__device__ __forceinline__ void load_chunk(const float* __restrict__ x, const ChunkItem& it,
                                           int64_t sb, float (&pa)[PF], float (&pb)[PF]) {
  const int lane = lane_id();
  const int64_t rem = it.m - sb;  // > 0 for an item's chunk
  const int64_t need = 2 * kWave * PF;
  const int nrec = (int)((rem < need ? rem : need) * 4);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(x + it.base + sb), 0, nrec, 0x00020000);
  const int voff = 8 * lane;
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    // per-lane offset in a register, the row offset as a scalar offset
    const int soff = 2 * kWave * i * 4;
    pa[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
    pb[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff + 4, soff, 0));
  }
}

template <int W, int D, int R>
__global__ __launch_bounds__(256) void sketch_fast_kernel(
    const float* __restrict__ x, const int64_t* __restrict__ x_off, int64_t N, FilterArgs fa,
    uint64_t* __restrict__ bits, const int64_t* __restrict__ bit_word_off,
    int32_t* __restrict__ nbits_out, unsigned long long* repair_count, int* err) {
  constexpr int SUB = kWave * R;          // windows per chunk
  constexpr int XCAP = (SUB - 1) * D + W; // samples a chunk's windows touch
  constexpr int SPAN = D * (R - 1) + W;   // samples of one lane's R windows
  constexpr int NP = (SPAN + 1) / 2;      // fp16 pairs a lane holds
  constexpr int PE = (W + 1) / 2;         // pairs of an even-aligned window
  constexpr int PO = W / 2 + 1;           // pairs of an odd-aligned window
  constexpr int NPAIR = XCAP / 2 + 2;     // pairs per copy (sample XCAP included)
  constexpr int PF = (NPAIR + kWave - 1) / kWave;
  constexpr int QCAP = SUB + kWave;
  static_assert(R <= 32, "R bits per lane must fit a word");

  __shared__ uint32_t ev[kWavesPerBlock][PF * kWave];
  __shared__ uint32_t od[kWavesPerBlock][PF * kWave];
  __shared__ uint32_t qser[kWavesPerBlock][QCAP];
  __shared__ uint32_t qwin[kWavesPerBlock][QCAP];
  __shared__ uint32_t bw[kWavesPerBlock][2 * R];
  __shared__ int qn[kWavesPerBlock];
  // fp16 filter pairs (even[p], odd[p]) side by side: read with a uniform
  // address at the point of use rather than held in scalar registers across
  // the whole loop
  __shared__ uint2 filt[(PE > PO ? PE : PO)];

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int lane = lane_id();
  RepairQueue q{qser[w], qwin[w], &qn[w]};
  uint32_t* bits32 = reinterpret_cast<uint32_t*>(bits);
  for (int p = threadIdx.x; p < (PE > PO ? PE : PO); p += blockDim.x)
    filt[p] = make_uint2(fa.even[p], fa.odd[p]);
  if (lane == 0) qn[w] = 0;
  __syncthreads();

  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t s0 = (int64_t)blockIdx.x * kWavesPerBlock + w;
  ChunkItem cur;
  cur.s = N;
  if (s0 < N) {
    cur = series_item<W, D>(s0, x_off, bit_word_off, nbits_out, err);
    if (cur.nb == 0) cur = next_item<W, D, SUB>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
  }
  float pa[PF], pb[PF];
  if (cur.s < N) load_chunk<PF>(x, cur, (int64_t)cur.c * SUB * D, pa, pb);

  while (cur.s < N) {
    // stage the chunk as fp16 pairs; flag it when a sample it uses could
    // overflow the fp16 products or is not finite
    bool bad = false;
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int p = lane + kWave * i;
      // x[2p-1]: the lane before's x[2p+1]; for lane 0, lane 63's of the previous pair
      // row (both shuffles run on the whole wave before the select)
      const float up = __shfl_up(pb[i], 1, kWave);
      const float last = i == 0 ? 0.0f : __shfl(pb[i == 0 ? 0 : i - 1], kWave - 1, kWave);
      const float prev = lane == 0 ? last : up;
      ev[w][p] = __builtin_bit_cast(uint32_t, pack_h2(pa[i], pb[i]));
      od[w][p] = __builtin_bit_cast(uint32_t, pack_h2(prev, pa[i]));
      bad |= (2 * p <= XCAP && !(__builtin_fabsf(pa[i]) < 16384.0f)) ||
             (2 * p + 1 <= XCAP && !(__builtin_fabsf(pb[i]) < 16384.0f));
    }
    const bool unsafe = ballot64(bad) != 0;
    if (lane < 2 * R) bw[w][lane] = 0;
    wave_sync_lds();

    // start loading the next chunk; it is consumed at the top of the next iteration
    const ChunkItem nxt = next_item<W, D, SUB>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
    if (nxt.s < N) load_chunk<PF>(x, nxt, (int64_t)nxt.c * SUB * D, pa, pb);

    const int nb = cur.nb;
    const int c = cur.c;
    const int wl = lane * R;
    const int nvalid = nb - c * SUB - wl;
    if (nvalid > 0) {
      const int a = wl * D;  // first sample of the lane's span
      const uint32_t* src = (a & 1) ? od[w] + (a + 1) / 2 : ev[w] + a / 2;
      h2 pr[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) pr[p] = as_h2(src[p]);
      float E = 0.0f;
#pragma unroll
      for (int p = 0; p < NP; ++p) E = fdot2(pr[p], pr[p], E);
      const float M = window_margin(fa, E, 2 * NP);
      float acc[R];
#pragma unroll
      for (int rho = 0; rho < R; ++rho) acc[rho] = 0.0f;
#pragma unroll
      for (int p = 0; p < (PE > PO ? PE : PO); ++p) {
        const uint2 f = filt[p];
#pragma unroll
        for (int rho = 0; rho < R; ++rho) {
          if (((D * rho) & 1) == 0) {
            if (p < PE) acc[rho] = fdot2(pr[(D * rho) / 2 + p], as_h2(f.x), acc[rho]);
          } else {
            if (p < PO) acc[rho] = fdot2(pr[(D * rho - 1) / 2 + p], as_h2(f.y), acc[rho]);
          }
        }
        if ((p & 7) == 7) asm volatile("" ::: "memory");
      }
      uint32_t mybits = 0, myflags = 0;
#pragma unroll
      for (int rho = 0; rho < R; ++rho) {
        if (rho < nvalid) {
          const bool flag = unsafe || !(__builtin_fabsf(acc[rho]) >= M);
          if (flag) myflags |= 1u << rho;
          else if (acc[rho] >= 0.0f) mybits |= 1u << rho;
        }
      }
      or_bits<R>(bw[w], wl, mybits);
      push_flags<R>(q, myflags, (uint32_t)cur.s, (uint32_t)(c * SUB + wl));
    }
    wave_sync_lds();
    const int nwords = (nb + 63) / 64;
    if (lane < 2 * R) {
      const int64_t wd = (int64_t)c * R + (lane >> 1);
      if (wd < nwords) bits32[2 * (cur.wo + wd) + (lane & 1)] = bw[w][lane];
    }
    while (qn[w] >= kWave) repair_round(fa, x, x_off, bits32, bit_word_off, q, repair_count);
    cur = nxt;
  }
  while (qn[w] > 0) repair_round(fa, x, x_off, bits32, bit_word_off, q, repair_count);
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
      while (*qcount >= kWave) repair_round(fa, x, x_off, bits32, bit_word_off, q, repair_count);
    }
  }
  while (*qcount > 0) repair_round(fa, x, x_off, bits32, bit_word_off, q, repair_count);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static uint16_t to_half_bits(float f) {
  _Float16 h = (_Float16)f;  // round to nearest even
  return __builtin_bit_cast(uint16_t, h);
}

static float round_up_f32(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

static ssh_status make_filter_args(const float* r, int W, int delta, FilterArgs& fa) {
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
    fa.odd[p] = (uint32_t)to_half_bits(rk(2 * p - 1)) | ((uint32_t)to_half_bits(rk(2 * p)) << 16);
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

// Workgroups for the fast path: as many as the device holds at once (every
// wavefront then walks many series and its repair queue drains in full
// rounds, with no second, partly filled round of workgroups), and no more
// than the series need.
static unsigned resident_grid(const void* kernel, int64_t N) {
  int dev = 0, cus = 0, per_cu = 0;
  unsigned cap = 2048;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) == hipSuccess &&
      cus > 0 && per_cu > 0)
    cap = (unsigned)(cus * per_cu);
  return grid_for(N, kWavesPerBlock, cap);
}

ssh_status sketch_launch(const float* x, const int64_t* x_off, int64_t N, const float* r, int W,
                         int delta, uint64_t* bits, const int64_t* bit_word_off, int32_t* nbits,
                         uint64_t* repair_count, hipStream_t stream, bool force_generic) {
  FilterArgs fa;
  ssh_status st = make_filter_args(r, W, delta, fa);
  if (st != SSH_OK) return st;
  if (N == 0) return SSH_OK;
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_sketch_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_sketch: cannot resolve error flag");
  unsigned long long* rc = reinterpret_cast<unsigned long long*>(repair_count);
  const unsigned grid = grid_for(N, kWavesPerBlock, 1 << 16);
  const dim3 blk(256);
#define SSH_FAST(WW, DD, RR)                                                                   \
  if (!force_generic && W == WW && delta == DD) {                                              \
    const unsigned fgrid = resident_grid(reinterpret_cast<const void*>(                        \
        &sketch_fast_kernel<WW, DD, RR>), N);                                                  \
    sketch_fast_kernel<WW, DD, RR><<<fgrid, blk, 0, stream>>>(x, x_off, N, fa, bits,          \
                                                              bit_word_off, nbits, rc, err);  \
    return check_launch("ssh_sketch");                                                         \
  }
  SSH_FAST(80, 3, 5)
  SSH_FAST(64, 4, 2)
  SSH_FAST(128, 4, 8)
  SSH_FAST(30, 5, 4)
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
