// Banded DTW re-rank (Section 2.1; the top-k step closing Algorithm 2).
//
// D(i,j) = (q_i - x_j)^2 + min(D(i-1,j), D(i,j-1), D(i-1,j-1)), D(0,0) = cost,
// cells with |i - j| > r or outside the matrix at +inf; distance = sqrt(D(lq-1, lx-1)).
// Every (query, candidate) pair has its own lengths lq, lx and its own
// Sakoe-Chiba radius r = floor(band_frac * max(lq, lx)).
//
// Planning.  The pairs of a call are sorted into classes by the lane width G
// their band needs (the smallest G of the instantiated set with 16 G >= 2 r + 2;
// pairs without a warping path, |lq - lx| > r, get +inf at once).  Three small
// kernels do it without atomics on global memory: per-workgroup class counts,
// one workgroup scanning them, and a scatter that lists every pair in slot
// order inside its class (one workgroup does all three for a small call).
// Three DTW launches, one per group of lane widths, then walk the lists, four
// pairs of one class per wavefront; wavefronts past their group's pairs exit
// at once.
//
// Layout of one pair: a 16-lane DPP row.  Lane L of the row owns G
// consecutive band offsets o = j - i = -r + L*G + g (g = 0..G-1) and walks
// the query rows, lane L handling row i = T - L at step T (a skew of one row
// per lane).  Within a lane the G cells of a row are computed left to right,
// each from its left neighbour (just computed), the cell above (the same
// lane's previous row at offset o+1) and the diagonal (previous row, same
// offset).  The two values a lane needs from its neighbours travel by DPP row
// shifts: the left of slot 0 from lane L-1 (which finished row i one step
// earlier) and the upper cell of slot G-1 from lane L+1 (whose slot 0 of row
// i-1 is computed first in this step).  Row ends yield +inf through the DPP
// bound, which is the band edge (-r-1) on the left; on the right the first
// offset past the band (r+1) is held at +inf.  The x values of a lane's G
// cells shift by one slot per row, so a lane loads one new x per row; in the
// steady state the ring of x registers is renamed by unrolling G rows instead
// of moved.
//
// Each cell costs one subtract, one three-way min, one fused multiply-add and
// one add of a per-slot constant in float32: the constant is +inf for the one
// slot that holds the first offset past the band (offset r + 1) and 0 for every
// other slot, which keeps that slot at +inf without a select (all cell values
// are >= 0, so adding 0 is exact).  In the steady state, blocks of rows whose
// x indices are provably inside the series on every lane load x unchecked,
// and each block's q and x values are loaded one block ahead.
//
// Early abandoning (the pruned re-rank's second pass).  After lane L has
// finished row T - L, the cells the row's lanes hold form a staircase that
// every warping path crosses, and the values along a path never decrease, so
// their minimum bounds the final total from below.  A wavefront whose four
// pairs all have that minimum above their cut stops and reports +inf.
#include <cmath>
#include <mutex>

#include "common.hpp"

namespace ssh {

constexpr float kInf = __builtin_inff();
constexpr int kSegLanes = 16;
constexpr int kPrologue = kSegLanes - 1;
constexpr int kNumG = 16;          // instantiated lane widths, see band_class
constexpr int kPlanSlots = 1024;   // pairs per planning workgroup (256 threads x 4)
constexpr uint8_t kNoDp = 0xFF;    // planning class of a pair that needs no DTW launch

// Lane-width class of a band of radius r: the index of the smallest G in
// {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 26, 28, 32} with 16 G >= 2 r + 2
// (band offsets plus the +inf guard offset), or -1 when r > SSH_MAX_BAND.
__host__ __device__ inline int band_class(int64_t r) {
  if (r < 0 || r > SSH_MAX_BAND) return -1;
  const int need = 2 * (int)r + 2;
  int c = 0;
#define SSH_CLS(GG)                     \
  if (need <= kSegLanes * (GG)) return c; \
  ++c;
  SSH_CLS(2) SSH_CLS(3) SSH_CLS(4) SSH_CLS(5) SSH_CLS(6) SSH_CLS(7) SSH_CLS(8) SSH_CLS(10)
  SSH_CLS(12) SSH_CLS(14) SSH_CLS(16) SSH_CLS(20) SSH_CLS(24) SSH_CLS(26) SSH_CLS(28) SSH_CLS(32)
#undef SSH_CLS
  return -1;
}

// Sakoe-Chiba radius of a pair: floor(band_frac * max(lq, lx)), the product
// taken in float64 (exact for lengths below 2^29).
__device__ __forceinline__ int64_t pair_radius(float band_frac, int64_t lq, int64_t lx) {
  const int64_t mx = lq > lx ? lq : lx;
  return (int64_t)floor((double)band_frac * (double)mx);
}

// Squared-distance cut of the pruned re-rank for a pair of lengths lq, lx,
// given tau, the largest first-pass distance of its query.  The float32 DTW
// total of a path of P <= lq + lx - 1 cells is at least (1 - 2^-24)^(P + 2)
// times the exact one, the float32 LB at most (1 + 2^-24)^(lx + 4) times the
// exact LB, and tau^2 recomputed from the rounded square root is within 9
// ulps of the total it came from; the factor is twice their sum, plus 2^-19
// so that the rounded distances differ strictly.  +inf when tau is +inf.
__device__ __forceinline__ float prune_cut(float tau, int64_t lq, int64_t lx) {
  const double m = (double)(lq + 2 * lx + 64) * 0x1p-23 + 0x1p-19;
  float f = (float)(1.0 + m);
  if ((double)f < 1.0 + m)  // the next float up (f is positive and finite)
    f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u);
  return tau * tau * f;
}

__device__ __forceinline__ float dpp_from_left(float v) {  // lane k <- lane k-1 of its row
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, kInf), __builtin_bit_cast(int, v),
                                         0x111, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane k <- lane k+1 of its row
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, kInf), __builtin_bit_cast(int, v),
                                         0x101, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ float dpp_min(float v) {
  return fminf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                                __builtin_bit_cast(int, v),
                                                __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false)));
}
// minimum over the 16 lanes of each DPP row (quad swaps, then rotations by 4 and 8)
__device__ __forceinline__ float row_min(float v) {
  v = dpp_min<0xB1>(v);
  v = dpp_min<0x4E>(v);
  v = dpp_min<0x124>(v);
  return dpp_min<0x128>(v);
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int t = __shfl_xor(v, o, kWave);
    v = t > v ? t : v;
  }
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int t = __shfl_xor(v, o, kWave);
    v = t < v ? t : v;
  }
  return v;
}

struct DtwLane {
  const float* qs;  // query values
  const float* xs;  // candidate values
  int lq, lx;
  int L;            // lane in its row
  int jn;           // x index of slot G-1 for the next row
};

__device__ __forceinline__ float x_at(const DtwLane& d, int j) {
  const int jc = j < 0 ? 0 : (j >= d.lx ? d.lx - 1 : j);
  const float v = d.xs[jc];
  return (unsigned)j < (unsigned)d.lx ? v : kInf;
}

// One row step with an explicit shift of the x ring; rows outside [0, lq)
// leave the lane's state untouched.
template <int G>
__device__ __forceinline__ void step_masked(DtwLane& d, float (&V)[G], float (&xr)[G], int T,
                                            const float (&cb)[G]) {
  const int i = T - d.L;
  const bool active = (unsigned)i < (unsigned)d.lq;
  const int ic = i < 0 ? 0 : (i >= d.lq ? d.lq - 1 : i);
  const float qv = d.qs[ic];
  float nv[G];
  const float leftN = dpp_from_left(V[G - 1]);
  float t = qv - xr[0];
  nv[0] = __builtin_fmaf(t, t, fminf(fminf(leftN, V[1]), V[0])) + cb[0];
#pragma unroll
  for (int g = 1; g < G - 1; ++g) {
    t = qv - xr[g];
    nv[g] = __builtin_fmaf(t, t, fminf(fminf(nv[g - 1], V[g + 1]), V[g])) + cb[g];
  }
  const float upN = dpp_from_right(active ? nv[0] : kInf);
  t = qv - xr[G - 1];
  nv[G - 1] = __builtin_fmaf(t, t, fminf(fminf(nv[G - 2], upN), V[G - 1])) + cb[G - 1];
#pragma unroll
  for (int g = 0; g < G; ++g) V[g] = active ? nv[g] : V[g];
#pragma unroll
  for (int g = 0; g < G - 1; ++g) xr[g] = xr[g + 1];
  xr[G - 1] = x_at(d, d.jn);
  d.jn += 1;
}

// Steady-state step: every lane's row is inside [0, lq).  Logical slot g is
// physical register (g + ROT) % G of the x ring.  The row's q value and the x
// value entering the ring were loaded one block of G steps earlier.
template <int G, int ROT>
__device__ __forceinline__ void step_full(DtwLane& d, float (&V)[G], float (&xr)[G], float qv,
                                          float xin, const float (&cb)[G]) {
  float nv[G];
  const float leftN = dpp_from_left(V[G - 1]);
  float t = qv - xr[(0 + ROT) % G];
  nv[0] = __builtin_fmaf(t, t, fminf(fminf(leftN, V[1]), V[0])) + cb[0];
#pragma unroll
  for (int g = 1; g < G - 1; ++g) {
    t = qv - xr[(g + ROT) % G];
    nv[g] = __builtin_fmaf(t, t, fminf(fminf(nv[g - 1], V[g + 1]), V[g])) + cb[g];
  }
  const float upN = dpp_from_right(nv[0]);
  t = qv - xr[(G - 1 + ROT) % G];
  nv[G - 1] = __builtin_fmaf(t, t, fminf(fminf(nv[G - 2], upN), V[G - 1])) + cb[G - 1];
#pragma unroll
  for (int g = 0; g < G; ++g) V[g] = nv[g];
  xr[ROT % G] = xin;
  d.jn += 1;
}

template <int G, int ROT>
__device__ __forceinline__ void steps_full(DtwLane& d, float (&V)[G], float (&xr)[G],
                                           const float (&qb)[G], const float (&xb)[G],
                                           const float (&cb)[G]) {
  if constexpr (ROT < G) {
    step_full<G, ROT>(d, V, xr, qb[ROT], xb[ROT], cb);
    steps_full<G, ROT + 1>(d, V, xr, qb, xb, cb);
  }
}

// The q values and incoming x values of the G steps from T0 (whose first x
// index is jn): x unchecked when IN (inside [0, lx) on every lane).
template <int G>
__device__ __forceinline__ void load_block(const DtwLane& d, int T0, int jn, bool in,
                                           float (&qb)[G], float (&xb)[G]) {
#pragma unroll
  for (int s = 0; s < G; ++s) qb[s] = d.qs[T0 + s - d.L];
  if (in) {
#pragma unroll
    for (int s = 0; s < G; ++s) xb[s] = d.xs[jn + s];
  } else {
#pragma unroll
    for (int s = 0; s < G; ++s) xb[s] = x_at(d, jn + s);
  }
}

// ---------------------------------------------------------------------------
// planning: class lists of the pairs to compute
// ---------------------------------------------------------------------------

// Pair of planning slot s: slot s itself, or plist[s] (-1: none).  Writes
// +inf for a pair that gets no DTW launch (no candidate in that column, an
// invalid id, an empty series, no warping path, a band wider than
// SSH_MAX_BAND) and returns its class otherwise.  A column past ncand gets
// +inf only when every slot is a pair (plist null).
__device__ __forceinline__ uint8_t plan_pair(int64_t s, const int32_t* __restrict__ plist,
                                             const int64_t* __restrict__ q_off,
                                             const int64_t* __restrict__ db_off, int64_t Ndb,
                                             const int64_t* __restrict__ cand,
                                             const int32_t* __restrict__ ncand, int C,
                                             float band_frac, float* __restrict__ dist, int* err) {
  const int64_t pair = plist != nullptr ? (int64_t)plist[s] : s;
  if (pair < 0) return kNoDp;
  const int64_t qi = pair / C;
  const int ci = (int)(pair - qi * C);
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  if (ci >= nc) {
    if (plist == nullptr) dist[pair] = kInf;
    return kNoDp;
  }
  const int64_t id = cand[pair];
  if (id < 0 || id >= Ndb) {
    atomicOr(err, 1);
    dist[pair] = kInf;
    return kNoDp;
  }
  const int64_t lq = q_off[qi + 1] - q_off[qi], lx = db_off[id + 1] - db_off[id];
  if (lq <= 0 || lx <= 0 || lq > (1 << 30) || lx > (1 << 30)) {
    if (lq < 0 || lx < 0 || lq > (1 << 30) || lx > (1 << 30)) atomicOr(err, 4);
    dist[pair] = kInf;
    return kNoDp;
  }
  const int64_t r = pair_radius(band_frac, lq, lx);
  const int64_t dl = lq - lx;
  if (dl > r || -dl > r) {
    dist[pair] = kInf;
    return kNoDp;
  }
  const int c = band_class(r);
  if (c < 0) {
    atomicOr(err, 2);
    dist[pair] = kInf;
    return kNoDp;
  }
  return (uint8_t)c;
}

// Per planning workgroup (kPlanSlots consecutive slots): the class of every
// slot and the number of slots in each class.
__global__ __launch_bounds__(256) void dtw_count_kernel(
    const int32_t* __restrict__ plist, int64_t nslots, const int64_t* __restrict__ q_off,
    const int64_t* __restrict__ db_off, int64_t Ndb, const int64_t* __restrict__ cand,
    const int32_t* __restrict__ ncand, int C, float band_frac, float* __restrict__ dist,
    uint8_t* __restrict__ cls, int32_t* __restrict__ bcnt, int* err) {
  __shared__ int cnt[kNumG];
  if (threadIdx.x < kNumG) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kPlanSlots;
#pragma unroll
  for (int j = 0; j < kPlanSlots / 256; ++j) {
    const int64_t s = b0 + j * 256 + threadIdx.x;
    if (s < nslots) {
      const uint8_t c = plan_pair(s, plist, q_off, db_off, Ndb, cand, ncand, C, band_frac, dist, err);
      cls[s] = c;
      if (c != kNoDp) atomicAdd(&cnt[c], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < kNumG) bcnt[(int64_t)blockIdx.x * kNumG + threadIdx.x] = cnt[threadIdx.x];
}

// One workgroup: each class's list is the concatenation, in workgroup order,
// of the planning workgroups' slots of that class; classes follow each other.
// boff[b][c] = where workgroup b's slots of class c start; seg[2c], seg[2c+1] =
// start and length of class c's list.
__global__ __launch_bounds__(1024) void dtw_scan_kernel(const int32_t* __restrict__ bcnt, int nblk,
                                                        int32_t* __restrict__ boff,
                                                        int32_t* __restrict__ seg) {
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t wpre[1024 / kWave];
  __shared__ uint32_t tot;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint32_t base = 0;
  for (int c = 0; c < kNumG; ++c) {
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 1024) {
      const int b = b0 + (int)threadIdx.x;
      const uint32_t v = b < nblk ? (uint32_t)bcnt[(int64_t)b * kNumG + c] : 0u;
      const uint32_t incl = wave_incl_scan(v);
      if (lane == kWave - 1) wsum[w] = incl;
      __syncthreads();
      if (w == 0) {
        const uint32_t t = lane < 1024 / kWave ? wsum[lane] : 0u;
        const uint32_t ti = wave_incl_scan(t);
        if (lane < 1024 / kWave) wpre[lane] = ti - t;
        if (lane == 1024 / kWave - 1) tot = ti;
      }
      __syncthreads();
      if (b < nblk) boff[(int64_t)b * kNumG + c] = (int32_t)(base + carry + wpre[w] + incl - v);
      carry += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      seg[2 * c] = (int32_t)base;
      seg[2 * c + 1] = (int32_t)carry;
    }
    base += carry;
  }
}

// Lists every slot with a class at its place: workgroup b's slots of class c,
// in slot order, from boff[b][c].  The entry is the pair index.
__global__ __launch_bounds__(256) void dtw_scatter_kernel(const uint8_t* __restrict__ cls,
                                                          const int32_t* __restrict__ plist,
                                                          int64_t nslots,
                                                          const int32_t* __restrict__ boff,
                                                          int32_t* __restrict__ list) {
  __shared__ int32_t run[kNumG];
  __shared__ int32_t wc[256 / kWave][kNumG];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x < kNumG) run[threadIdx.x] = boff[(int64_t)blockIdx.x * kNumG + threadIdx.x];
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kPlanSlots;
  for (int j = 0; j < kPlanSlots / 256; ++j) {
    const int64_t s = b0 + j * 256 + threadIdx.x;
    const int c = s < nslots ? (int)cls[s] : (int)kNoDp;
    int rank = 0;
    for (int cc = 0; cc < kNumG; ++cc) {
      const uint64_t m = ballot64(c == cc);
      if (lane == 0) wc[w][cc] = __builtin_popcountll(m);
      if (c == cc)
        rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    }
    __syncthreads();
    if (c != (int)kNoDp) {
      int pos = run[c] + rank;
      for (int v = 0; v < w; ++v) pos += wc[v][c];
      list[pos] = plist != nullptr ? plist[s] : (int32_t)s;
    }
    __syncthreads();
    if (threadIdx.x < kNumG) {
      int add = 0;
      for (int v = 0; v < 256 / kWave; ++v) add += wc[v][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// The three steps above in one workgroup, for calls of at most kSmallPlan
// pairs (a small query batch), with the same lists: classes and counts in
// LDS, the scan by one thread, then the scatter in slot order.
constexpr int kSmallPlan = 4096;
__global__ __launch_bounds__(1024) void dtw_plan_small_kernel(
    const int32_t* __restrict__ plist, int64_t nslots, const int64_t* __restrict__ q_off,
    const int64_t* __restrict__ db_off, int64_t Ndb, const int64_t* __restrict__ cand,
    const int32_t* __restrict__ ncand, int C, float band_frac, float* __restrict__ dist,
    int32_t* __restrict__ list, int32_t* __restrict__ seg, int* err) {
  __shared__ uint8_t cls[kSmallPlan];
  __shared__ int cnt[kNumG];
  __shared__ int run[kNumG];
  __shared__ int wc[1024 / kWave][kNumG];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x < kNumG) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t s = threadIdx.x; s < nslots; s += 1024) {
    const uint8_t c = plan_pair(s, plist, q_off, db_off, Ndb, cand, ncand, C, band_frac, dist, err);
    cls[s] = c;
    if (c != kNoDp) atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int b = 0;
    for (int c = 0; c < kNumG; ++c) {
      seg[2 * c] = b;
      seg[2 * c + 1] = cnt[c];
      run[c] = b;
      b += cnt[c];
    }
  }
  __syncthreads();
  for (int64_t s0 = 0; s0 < nslots; s0 += 1024) {
    const int64_t s = s0 + threadIdx.x;
    const int c = s < nslots ? (int)cls[s] : (int)kNoDp;
    int rank = 0;
    for (int cc = 0; cc < kNumG; ++cc) {
      const uint64_t m = ballot64(c == cc);
      if (lane == 0) wc[w][cc] = __builtin_popcountll(m);
      if (c == cc)
        rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    }
    __syncthreads();
    if (c != (int)kNoDp) {
      int pos = run[c] + rank;
      for (int v = 0; v < w; ++v) pos += wc[v][c];
      list[pos] = plist != nullptr ? plist[s] : (int32_t)s;
    }
    __syncthreads();
    if (threadIdx.x < kNumG) {
      int add = 0;
      for (int v = 0; v < 1024 / kWave; ++v) add += wc[v][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// DTW of the four pairs list[start + base .. + 4) of one class (lane width G),
// one pair per 16-lane row of the wavefront
// ---------------------------------------------------------------------------
template <int G, bool ABANDON>
__device__ __forceinline__ void dtw_wave(
    const float* __restrict__ q, const int64_t* __restrict__ q_off, const float* __restrict__ db,
    const int64_t* __restrict__ db_off, const int64_t* __restrict__ cand, int C, float band_frac,
    const int32_t* __restrict__ list, int start, int count, int64_t base,
    const float* __restrict__ tauq, float* __restrict__ dist) {
  static_assert(G >= 2, "at least two offsets per lane");
  const int lane = lane_id();
  const int L = lane & (kSegLanes - 1);
  {
    const int64_t slot = base + (lane >> 4);
    const bool own = slot < count;
    // a row past the end of the list repeats the wave's first pair (which
    // exists) and writes nothing, so every row reads valid memory
    const int pair = list[start + (own ? slot : base)];
    const int qi = pair / C;
    const int64_t id = cand[pair];
    const int64_t qa = q_off[qi], xa = db_off[id];
    DtwLane d;
    d.lq = (int)(q_off[qi + 1] - qa);
    d.lx = (int)(db_off[id + 1] - xa);
    d.qs = q + qa;
    d.xs = db + xa;
    d.L = L;
    const int r = (int)pair_radius(band_frac, d.lq, d.lx);
    const float cut = ABANDON ? prune_cut(tauq[qi], d.lq, d.lx) : kInf;
    const int span = 2 * r + 1;  // first offset past the band: -r + span
    const int Lv = span / G, gv = span % G;
    const int L0 = r / G, g0 = r % G;  // slot of offset 0 (holds D(-1,-1) = 0)
    // the first offset past the band (slot gv of lane Lv) stays +inf: its cost
    // gets +inf added; every other cell adds 0 (exact: all values are >= 0)
    float cb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) cb[g] = (L == Lv && g == gv) ? kInf : 0.0f;
    // At step T lane L is on row i = T - L; its x ring holds x[i + o] for its
    // G offsets o, so at T = 0 (row -L) it starts at x[L(G-1) - r + g].
    float V[G], xr[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      V[g] = (L == L0 && g == g0) ? 0.0f : kInf;
      xr[g] = x_at(d, L * (G - 1) - r + g);
    }
    d.jn = L * (G - 1) - r + G;  // slot G-1 of row -L + 1
    // wave-uniform loop bounds (held in scalar registers)
    const int Ttot = __builtin_amdgcn_readfirstlane(wave_max_i(d.lq)) + kPrologue;
    const int lqmin = __builtin_amdgcn_readfirstlane(wave_min_i(d.lq));
    bool abandoned = false;
    int T = 0;
    const int p_end = kPrologue < Ttot ? kPrologue : Ttot;
    for (; T < p_end; ++T) step_masked<G>(d, V, xr, T, cb);
    if (lqmin >= kPrologue) {
      const int full = (lqmin - kPrologue) / G * G;
      const int T_end = kPrologue + full;
      // At step T lane L loads x[T + L(G-1) - r + G].  Over a block of G
      // steps from T0 the indices span [T0 - r + G, T0 + 17G - 16 - r] (lanes 0
      // and 15), inside [0, min(lx, lq)) when T0 >= r - G and
      // T0 <= min(lx, lq) + 15 - 17G + r; the block loads unchecked when that
      // holds on every row of the wave.
      const int lmin = d.lx < d.lq ? d.lx : d.lq;
      const int in_lo = r - G;
      const int in_hi = lmin + (kSegLanes - 1) - (kSegLanes + 1) * G + r;  // last T0 allowed
      auto in_at = [&](int T0) { return ballot64(!(T0 >= in_lo && T0 <= in_hi)) == 0; };
      // each block's loads are issued one block ahead, while the previous
      // block computes, into two buffers in turn
      float qa_[G], xa_[G], qc_[G], xc_[G];
      if (kPrologue < T_end) load_block<G>(d, kPrologue, d.jn, in_at(kPrologue), qa_, xa_);
      for (int T0 = kPrologue; T0 < T_end; T0 += 2 * G) {
        const int T1 = T0 + G, T2 = T0 + 2 * G;
        if (T1 < T_end) load_block<G>(d, T1, d.jn + G, in_at(T1), qc_, xc_);
        steps_full<G, 0>(d, V, xr, qa_, xa_, cb);
        if (T1 >= T_end) break;
        if (T2 < T_end) load_block<G>(d, T2, d.jn + G, in_at(T2), qa_, xa_);
        steps_full<G, 0>(d, V, xr, qc_, xc_, cb);
        if constexpr (ABANDON) {
          float m = V[0];
#pragma unroll
          for (int g = 1; g < G; ++g) m = fminf(m, V[g]);
          if (ballot64(!(row_min(m) > cut)) == 0) {
            abandoned = true;
            break;
          }
        }
      }
      T = T_end;
    }
    if (!abandoned)
      for (; T < Ttot; ++T) step_masked<G>(d, V, xr, T, cb);

    // D(lq-1, lx-1) sits at offset lx - lq
    if (own) {
      const int of = d.lx - d.lq;
      if (!abandoned && of >= -r && of <= r) {
        const int Lf = (of + r) / G, gf = (of + r) % G;
        float res = kInf;
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (g == gf) res = V[g];
        if (L == Lf) dist[pair] = __builtin_sqrtf(res);
      } else if (L == 0) {
        dist[pair] = kInf;
      }
    }
  }
}

// Lane widths are launched in three groups, {2, ..., 8}, {10, ..., 16} and
// {20, ..., 32} (classes [0, 7), [7, 11), [11, 16)), so that a call costs
// three DTW launches whatever its lengths, while a narrow band does not run
// with the register budget of a wide one.  Wavefront w of a group takes four
// consecutive pairs of one class: the classes' lists are cut into quads in
// class order and w indexes the quads.
template <int CLS0, int NCLS, bool ABANDON>
__global__ __launch_bounds__(256) void dtw_group_kernel(
    const float* __restrict__ q, const int64_t* __restrict__ q_off, const float* __restrict__ db,
    const int64_t* __restrict__ db_off, const int64_t* __restrict__ cand, int C, float band_frac,
    const int32_t* __restrict__ list, const int32_t* __restrict__ seg,
    const float* __restrict__ tauq, float* __restrict__ dist) {
  int64_t w = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  int cls = -1, start = 0, count = 0;
#pragma unroll
  for (int c = CLS0; c < CLS0 + NCLS; ++c) {
    const int n = seg[2 * c + 1];
    const int64_t quads = (n + 3) / 4;
    if (cls < 0) {
      if (w < quads) {
        cls = c;
        start = seg[2 * c];
        count = n;
      } else {
        w -= quads;
      }
    }
  }
  if (cls < 0) return;
  const int64_t base = w * 4;
#define SSH_CASE(CC, GG)                                                                       \
  case CC:                                                                                     \
    dtw_wave<GG, ABANDON>(q, q_off, db, db_off, cand, C, band_frac, list, start, count, base, \
                          tauq, dist);                                                         \
    break;
  switch (cls) {
    SSH_CASE(0, 2) SSH_CASE(1, 3) SSH_CASE(2, 4) SSH_CASE(3, 5) SSH_CASE(4, 6) SSH_CASE(5, 7)
    SSH_CASE(6, 8) SSH_CASE(7, 10) SSH_CASE(8, 12) SSH_CASE(9, 14) SSH_CASE(10, 16)
    SSH_CASE(11, 20) SSH_CASE(12, 24) SSH_CASE(13, 26) SSH_CASE(14, 28) SSH_CASE(15, 32)
    default: break;
  }
#undef SSH_CASE
}

// ---------------------------------------------------------------------------
// per-query top-k by (distance, id)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ dist,
                                                   const int64_t* __restrict__ cand,
                                                   const int32_t* __restrict__ ncand, int C, int k,
                                                   int64_t* __restrict__ out_id,
                                                   float* __restrict__ out_dist) {
  __shared__ uint64_t a[SSH_MAX_C];
  const int qi = blockIdx.x;
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  int n2 = 1;
  while (n2 < C) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    uint64_t key = ~0ull;
    if (i < nc) {
      const float dv = dist[(int64_t)qi * C + i];
      key = ((uint64_t)__builtin_bit_cast(uint32_t, dv) << 32) |
            (uint32_t)cand[(int64_t)qi * C + i];
    }
    a[i] = key;
  }
  __syncthreads();
  for (int kk = 2; kk <= n2; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t x = a[i], y = a[p];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const uint64_t key = a[i];
    const bool ok = i < nc && key != ~0ull;
    out_id[(int64_t)qi * k + i] = ok ? (int64_t)(uint32_t)key : -1;
    out_dist[(int64_t)qi * k + i] = ok ? __builtin_bit_cast(float, (uint32_t)(key >> 32)) : kInf;
  }
}

// ---------------------------------------------------------------------------
// Lower bounds for pruning (Section 2.1: DTW is costly, so cheap bounds
// discard candidates first; Algorithm 2's re-rank relies on such pruning).
//
// LB_Kim: the first and the last cell lie on every warping path, so
//     LB_Kim = (q_0 - x_0)^2 + (q_{lq-1} - x_{lx-1})^2 <= D   (one term when
//     both lengths are 1).
// LB_Keogh: for candidate value x_j the query values it can be matched with
// are q_i, |i - j| <= r, so every warping path pays at least the squared
// distance from x_j to [min, max] of that window:
//     LB_Keogh = sum_j dist(x_j, [Lo_j, U_j])^2 <= D.
// The envelope (U, Lo) is built once per query with its own radius
// floor(band_frac * lq); it bounds the pairs whose candidate is not longer
// than the query (their radius is the same), the others take LB_Kim alone.
// A query's k candidates with the smallest bound are computed first; the
// largest of their distances, tau, bounds the k-th best, and a candidate is
// skipped when its bound exceeds tau^2 by more than every rounding involved
// can account for (prune_cut), which leaves its distance strictly above the
// k-th best: the top k are those of dtw_rerank.  The survivors' DTW abandons
// early against the same cut.
// ---------------------------------------------------------------------------

constexpr int kLbLds = 4096;   // query envelope values staged in LDS for the bounds
constexpr int kEnvJ = 256;     // envelope entries per workgroup round

__device__ __forceinline__ bool envelope_ok(const int64_t* __restrict__ q_off, int qi,
                                            float band_frac, int64_t env_cap) {
  const int64_t lq = q_off[qi + 1] - q_off[qi];
  return lq > 0 && lq <= (1 << 30) && q_off[qi + 1] <= env_cap &&
         pair_radius(band_frac, lq, lq) <= SSH_MAX_BAND;
}

// Envelope of each query over j in [0, lq): the window q[max(0, j - r),
// min(lq - 1, j + r)], r = floor(band_frac * lq), stored at the query's own
// offsets.  One workgroup per query, 256 consecutive j per round with the
// query values their windows cover (at most 256 + 2 SSH_MAX_BAND) staged in
// LDS.  A query past the workspace capacity raises flag 8 and gets no
// envelope (its pairs take LB_Kim).
__global__ __launch_bounds__(kEnvJ) void lb_envelope_kernel(const float* __restrict__ q,
                                                            const int64_t* __restrict__ q_off,
                                                            float band_frac, int64_t env_cap,
                                                            float* __restrict__ U,
                                                            float* __restrict__ Lo, int* err) {
  __shared__ float qsh[kEnvJ + 2 * SSH_MAX_BAND + 1];
  const int qi = blockIdx.x;
  const int64_t qa = q_off[qi];
  if (q_off[qi + 1] > env_cap) {
    if (threadIdx.x == 0) atomicOr(err, 8);
    return;
  }
  if (!envelope_ok(q_off, qi, band_frac, env_cap)) return;
  const int lq = (int)(q_off[qi + 1] - qa);
  const int r = (int)pair_radius(band_frac, lq, lq);
  const float* qs = q + qa;
  for (int j0 = 0; j0 < lq; j0 += kEnvJ) {
    const int s0 = j0 - r < 0 ? 0 : j0 - r;
    const int s1 = j0 + kEnvJ + r < lq ? j0 + kEnvJ + r : lq;  // staged q[s0, s1)
    __syncthreads();
    for (int i = s0 + (int)threadIdx.x; i < s1; i += kEnvJ) qsh[i - s0] = qs[i];
    __syncthreads();
    const int j = j0 + (int)threadIdx.x;
    if (j < lq) {
      const int a = j - r < 0 ? 0 : j - r;
      const int b = j + r < lq - 1 ? j + r : lq - 1;
      float mx = -kInf, mn = kInf;
      for (int i = a; i <= b; ++i) {
        const float v = qsh[i - s0];
        mx = fmaxf(mx, v);
        mn = fminf(mn, v);
      }
      U[qa + j] = mx;
      Lo[qa + j] = mn;
    }
  }
}

// Bound of every live pair (float32): max(LB_Kim, LB_Keogh) where the
// envelope applies, else LB_Kim.  One workgroup per query and four of its
// candidates, one wavefront each, the query's envelope in LDS when
// lq <= kLbLds.  A pair the DTW step will not compute (invalid id, empty
// series, no warping path) gets 0 and is left to that step.
__global__ __launch_bounds__(256) void lb_bound_kernel(
    const float* __restrict__ q, const int64_t* __restrict__ q_off, const float* __restrict__ db,
    const int64_t* __restrict__ db_off, int64_t Ndb, const int64_t* __restrict__ cand,
    const int32_t* __restrict__ ncand, int C, float band_frac, int64_t env_cap,
    const float* __restrict__ U, const float* __restrict__ Lo, float* __restrict__ lb) {
  __shared__ float env[2 * kLbLds];  // U then Lo when staged
  const int groups = (C + 3) / 4;
  const int qi = blockIdx.x / groups;
  const int c0 = (blockIdx.x - qi * groups) * 4;
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  if (c0 >= nc) return;  // no candidate here (uniform over the workgroup)
  const int64_t qa = q_off[qi];
  const int64_t lq = q_off[qi + 1] - qa;
  const bool eok = envelope_ok(q_off, qi, band_frac, env_cap);
  const float* u = U + qa;
  const float* lo = Lo + qa;
  if (eok && lq <= kLbLds) {
    for (int j = threadIdx.x; j < lq; j += blockDim.x) {
      env[j] = u[j];
      env[kLbLds + j] = lo[j];
    }
    u = env;
    lo = env + kLbLds;
  }
  __syncthreads();
  const int ci = c0 + threadIdx.x / kWave;
  if (ci >= nc) return;
  const int64_t pair = (int64_t)qi * C + ci;
  const int64_t id = cand[pair];
  float s = 0.0f;
  if (id >= 0 && id < Ndb && lq > 0 && lq <= (1 << 30)) {
    const int64_t lx = db_off[id + 1] - db_off[id];
    if (lx > 0 && lx <= (1 << 30)) {
      const float* xs = db + db_off[id];
      const float* qs = q + qa;
      if (eok && lx <= lq) {
        for (int64_t j = lane_id(); j < lx; j += kWave) {
          const float x = xs[j];
          const float t = x > u[j] ? x - u[j] : (x < lo[j] ? lo[j] - x : 0.0f);
          s = __builtin_fmaf(t, t, s);
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
      }
      const float d0 = qs[0] - xs[0];
      float kim = d0 * d0;
      if (lq > 1 || lx > 1) {
        const float d1 = qs[lq - 1] - xs[lx - 1];
        kim = kim + d1 * d1;
      }
      s = fmaxf(s, kim);
    }
  }
  if (lane_id() == 0) lb[pair] = s;
}

// Per query: distances preset to +inf; the k live candidates with the
// smallest bound (ties by column) marked 1 and listed in the first pass's
// slots list1[qi k ..) (-1 past the live count), the other live candidates
// marked 2, the rest 0.
__global__ __launch_bounds__(256) void lb_select_kernel(const float* __restrict__ lb,
                                                        const int32_t* __restrict__ ncand, int C,
                                                        int k, uint8_t* __restrict__ mark,
                                                        float* __restrict__ dist,
                                                        int32_t* __restrict__ list1) {
  __shared__ uint64_t a[SSH_MAX_C];
  const int qi = blockIdx.x;
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  int n2 = 1;
  while (n2 < (nc > 0 ? nc : 1)) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x)
    a[i] = i < nc ? ((uint64_t)__builtin_bit_cast(uint32_t, lb[(int64_t)qi * C + i]) << 32) | (uint32_t)i
                  : ~0ull;
  for (int i = threadIdx.x; i < C; i += blockDim.x) {
    mark[(int64_t)qi * C + i] = i < nc ? 2 : 0;
    dist[(int64_t)qi * C + i] = kInf;
  }
  __syncthreads();
  for (int kk = 2; kk <= n2; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t x = a[i], y = a[p];
          const bool up = (i & kk) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const int first = nc < k ? nc : k;
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    if (t < first) {
      const int ci = (int)(uint32_t)a[t];
      mark[(int64_t)qi * C + ci] = 1;
      list1[(int64_t)qi * k + t] = (int32_t)((int64_t)qi * C + ci);
    } else {
      list1[(int64_t)qi * k + t] = -1;
    }
  }
}

// Per query, after the first pass: tau = the largest first-pass distance
// (kept in tauq for the second pass's early abandoning); the candidates
// marked 2 whose bound does not exceed their cut fill the second pass's
// slots list2[qi (C - k) ..), the rest of which get -1 (a dropped candidate
// keeps its +inf distance).  A candidate with an invalid id is kept, so that
// the DTW step reports it.
__global__ __launch_bounds__(256) void lb_prune_kernel(
    const float* __restrict__ lb, const float* __restrict__ dist, const int64_t* __restrict__ q_off,
    const int64_t* __restrict__ db_off, int64_t Ndb, const int64_t* __restrict__ cand,
    const int32_t* __restrict__ ncand, int C, int k, const uint8_t* __restrict__ mark,
    float* __restrict__ tauq, int32_t* __restrict__ list2) {
  __shared__ float tmax[256 / kWave];
  __shared__ uint32_t nkeep;
  const int qi = blockIdx.x;
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  if (threadIdx.x == 0) nkeep = 0;
  float t = -kInf;
  for (int i = threadIdx.x; i < nc; i += blockDim.x)
    if (mark[(int64_t)qi * C + i] == 1) t = fmaxf(t, dist[(int64_t)qi * C + i]);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) t = fmaxf(t, __shfl_xor(t, o, kWave));
  if (lane_id() == 0) tmax[threadIdx.x / kWave] = t;
  __syncthreads();
  float tau = -kInf;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tau = fmaxf(tau, tmax[w]);
  if (threadIdx.x == 0) tauq[qi] = tau;
  const int64_t lq = q_off[qi + 1] - q_off[qi];
  int32_t* l2 = list2 + (int64_t)qi * (C - k);
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int64_t p = (int64_t)qi * C + i;
    if (mark[p] != 2) continue;
    const int64_t id = cand[p];
    bool keep = true;
    if (id >= 0 && id < Ndb) {
      const int64_t lx = db_off[id + 1] - db_off[id];
      keep = !(lb[p] > prune_cut(tau, lq, lx));
    }
    if (keep) l2[atomicAdd(&nkeep, 1u)] = (int32_t)p;
  }
  __syncthreads();
  for (int i = (int)nkeep + threadIdx.x; i < C - k; i += blockDim.x) l2[i] = -1;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
__device__ int g_dtw_err;

int take_dtw_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_dtw_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_dtw_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

static inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Planning scratch for nslots pairs: classes (u8), the class lists (i32),
// per-workgroup counts and offsets, and the class segments.
static inline int64_t plan_blocks(int64_t nslots) { return ceil_div(nslots, kPlanSlots); }
static size_t plan_bytes(int64_t nslots) {
  const int64_t nb = plan_blocks(nslots);
  return al256((size_t)nslots) + al256((size_t)nslots * 4) + 2 * al256((size_t)nb * kNumG * 4) +
         al256(2 * kNumG * 4);
}

struct PlanWs {
  uint8_t* cls;
  int32_t* list;
  int32_t* bcnt;
  int32_t* boff;
  int32_t* seg;
};

static PlanWs plan_carve(char* p, int64_t nslots) {
  const int64_t nb = plan_blocks(nslots);
  PlanWs w;
  w.cls = reinterpret_cast<uint8_t*>(p);
  p += al256((size_t)nslots);
  w.list = reinterpret_cast<int32_t*>(p);
  p += al256((size_t)nslots * 4);
  w.bcnt = reinterpret_cast<int32_t*>(p);
  p += al256((size_t)nb * kNumG * 4);
  w.boff = reinterpret_cast<int32_t*>(p);
  p += al256((size_t)nb * kNumG * 4);
  w.seg = reinterpret_cast<int32_t*>(p);
  return w;
}

struct DtwArgs {
  const float* q;
  const int64_t* q_off;
  const float* db;
  const int64_t* db_off;
  int64_t Ndb;
  const int64_t* cand;
  const int32_t* ncand;
  int C;
  float band_frac;
  int* err;
};

// One wavefront per four listed pairs of a class: a group's classes hold at
// most nslots pairs, plus one partial quad per class; wavefronts past the
// group's quads exit at once.
template <int CLS0, int NCLS>
static void launch_group(int64_t nslots, const DtwArgs& a, const PlanWs& pw, const float* tauq,
                         float* dist, hipStream_t s) {
  const unsigned grid = (unsigned)ceil_div(ceil_div(nslots, 4) + NCLS, 4);
  if (tauq != nullptr)
    dtw_group_kernel<CLS0, NCLS, true><<<grid, 256, 0, s>>>(
        a.q, a.q_off, a.db, a.db_off, a.cand, a.C, a.band_frac, pw.list, pw.seg, tauq, dist);
  else
    dtw_group_kernel<CLS0, NCLS, false><<<grid, 256, 0, s>>>(
        a.q, a.q_off, a.db, a.db_off, a.cand, a.C, a.band_frac, pw.list, pw.seg, tauq, dist);
}

// Distances of the nslots pairs of plist (every pair of the [nq][C] grid when
// plist is null): planning, then one launch per lane width.
static ssh_status run_dtw(hipStream_t s, const DtwArgs& a, const int32_t* plist, int64_t nslots,
                          const float* tauq, float* dist, char* plan_ws) {
  if (nslots == 0) return SSH_OK;
  const PlanWs pw = plan_carve(plan_ws, nslots);
  if (nslots <= kSmallPlan) {
    dtw_plan_small_kernel<<<1, 1024, 0, s>>>(plist, nslots, a.q_off, a.db_off, a.Ndb, a.cand,
                                             a.ncand, a.C, a.band_frac, dist, pw.list, pw.seg,
                                             a.err);
  } else {
    const int64_t nb = plan_blocks(nslots);
    dtw_count_kernel<<<(unsigned)nb, 256, 0, s>>>(plist, nslots, a.q_off, a.db_off, a.Ndb,
                                                  a.cand, a.ncand, a.C, a.band_frac, dist, pw.cls,
                                                  pw.bcnt, a.err);
    dtw_scan_kernel<<<1, 1024, 0, s>>>(pw.bcnt, (int)nb, pw.boff, pw.seg);
    dtw_scatter_kernel<<<(unsigned)nb, 256, 0, s>>>(pw.cls, plist, nslots, pw.boff, pw.list);
  }
  launch_group<0, 7>(nslots, a, pw, tauq, dist, s);
  launch_group<7, 4>(nslots, a, pw, tauq, dist, s);
  launch_group<11, 5>(nslots, a, pw, tauq, dist, s);
  return check_launch("dtw_rerank");
}

// Fills the launch arguments once the host-side checks have passed (the
// error flag's address is the first device query of a call).
static ssh_status dtw_args(DtwArgs& a, const float* q, const int64_t* q_off, const float* db,
                           const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                           const int32_t* ncand, int C, float band_frac, const char* what) {
  a = DtwArgs{q, q_off, db, db_off, Ndb, cand, ncand, C, band_frac, nullptr};
  if (hipGetSymbolAddress((void**)&a.err, HIP_SYMBOL(g_dtw_err)) != hipSuccess)
    return fail(SSH_EDEVICE, std::string(what) + ": cannot resolve error flag");
  return SSH_OK;
}

// Workspace of the plain re-rank: distances [nq][C] (float32), then the
// planning scratch for nq C pairs.
size_t rerank_workspace_bytes(int nq, int C) {
  const int64_t pc = (int64_t)nq * C;
  return al256((size_t)pc * 4) + plan_bytes(pc);
}

ssh_status rerank_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                         const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                         const int32_t* ncand, int C, float band_frac, int k, int64_t* out_id,
                         float* out_dist, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nq == 0) return SSH_OK;
  if ((int64_t)nq * C > INT32_MAX) return fail(SSH_EUNSUPPORTED, "dtw_rerank: nq * C above 2^31 - 1");
  if (ws_bytes < rerank_workspace_bytes(nq, C)) return fail(SSH_EINVAL, "dtw_rerank: workspace too small");
  DtwArgs a;
  ssh_status st = dtw_args(a, q, q_off, db, db_off, Ndb, cand, ncand, C, band_frac, "dtw_rerank");
  if (st != SSH_OK) return st;
  const int64_t pc = (int64_t)nq * C;
  char* p = static_cast<char*>(ws);
  float* dist = reinterpret_cast<float*>(p);
  st = run_dtw(stream, a, nullptr, pc, nullptr, dist, p + al256((size_t)pc * 4));
  if (st != SSH_OK) return st;
  topk_kernel<<<nq, 256, 0, stream>>>(dist, cand, ncand, C, k, out_id, out_dist);
  return check_launch("dtw_rerank");
}

// Workspace of the pruned re-rank: distances and bounds [nq][C] (float32),
// marks [nq][C] (u8), the two passes' slot lists (nq k, then nq (C - k),
// int32), tau per query, the planning scratch for nq C pairs, then the query
// envelopes U and Lo (q_values float32 each, at the queries' offsets).
static size_t rerank_lb_fixed_bytes(int nq, int C) {
  const size_t pc = (size_t)nq * C;
  return 3 * al256(pc * 4) + al256(pc) + al256((size_t)nq * 4) + plan_bytes((int64_t)pc);
}

size_t rerank_lb_workspace_bytes(int nq, int C, int64_t q_values) {
  return rerank_lb_fixed_bytes(nq, C) + 2 * al256((size_t)q_values * 4);
}

ssh_status rerank_lb_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                            const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                            const int32_t* ncand, int C, float band_frac, int k, int64_t* out_id,
                            float* out_dist, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (nq == 0) return SSH_OK;
  if ((int64_t)nq * C > INT32_MAX)
    return fail(SSH_EUNSUPPORTED, "dtw_rerank_lb: nq * C above 2^31 - 1");
  const size_t fixed = rerank_lb_fixed_bytes(nq, C);
  if (ws_bytes < fixed + 512) return fail(SSH_EINVAL, "dtw_rerank_lb: workspace too small");
  DtwArgs a;
  ssh_status st = dtw_args(a, q, q_off, db, db_off, Ndb, cand, ncand, C, band_frac,
                           "dtw_rerank_lb");
  if (st != SSH_OK) return st;
  const size_t pc = (size_t)nq * C;
  char* p = static_cast<char*>(ws);
  float* dist = reinterpret_cast<float*>(p);
  p += al256(pc * 4);
  float* lb = reinterpret_cast<float*>(p);
  p += al256(pc * 4);
  uint8_t* mark = reinterpret_cast<uint8_t*>(p);
  p += al256(pc);
  int32_t* list1 = reinterpret_cast<int32_t*>(p);  // nq k slots
  int32_t* list2 = list1 + (size_t)nq * k;          // nq (C - k) slots
  p += al256(pc * 4);
  float* tauq = reinterpret_cast<float*>(p);
  p += al256((size_t)nq * 4);
  char* plan_ws = p;
  p += plan_bytes((int64_t)pc);
  // the rest holds the two envelopes, each of env_cap values
  const size_t half = ((ws_bytes - fixed) / 2) & ~(size_t)255;
  const int64_t env_cap = (int64_t)(half / 4);
  float* U = reinterpret_cast<float*>(p);
  float* Lo = reinterpret_cast<float*>(p + half);
  lb_envelope_kernel<<<nq, kEnvJ, 0, stream>>>(q, q_off, band_frac, env_cap, U, Lo, a.err);
  lb_bound_kernel<<<(unsigned)((int64_t)nq * ((C + 3) / 4)), 256, 0, stream>>>(
      q, q_off, db, db_off, Ndb, cand, ncand, C, band_frac, env_cap, U, Lo, lb);
  lb_select_kernel<<<nq, 256, 0, stream>>>(lb, ncand, C, k, mark, dist, list1);
  st = check_launch("dtw_rerank_lb");
  if (st != SSH_OK) return st;
  st = run_dtw(stream, a, list1, (int64_t)nq * k, nullptr, dist, plan_ws);
  if (st != SSH_OK) return st;
  if (C > k) {
    lb_prune_kernel<<<nq, 256, 0, stream>>>(lb, dist, q_off, db_off, Ndb, cand, ncand, C, k, mark,
                                            tauq, list2);
    st = run_dtw(stream, a, list2, (int64_t)nq * (C - k), tauq, dist, plan_ws);
    if (st != SSH_OK) return st;
  }
  topk_kernel<<<nq, 256, 0, stream>>>(dist, cand, ncand, C, k, out_id, out_dist);
  return check_launch("dtw_rerank_lb");
}

// ---------------------------------------------------------------------------
// Allocation-free re-rank: the workspace of dtw_rerank in a static array
// ---------------------------------------------------------------------------
// One copy per device, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address is resolved once per device with
// hipGetSymbolAddress and every launch takes that address.
constexpr size_t kNoAllocScratch = SSH_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static ssh_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SSH_EDEVICE, "dtw_rerank_noalloc: no current device");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SSH_EUNSUPPORTED, "dtw_rerank_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(SSH_EDEVICE, std::string("dtw_rerank_noalloc: cannot resolve the scratch array: ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SSH_OK;
}

ssh_status rerank_noalloc_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                                 const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                                 const int32_t* ncand, int C, float band_frac, int k,
                                 int64_t* out_id, float* out_dist, hipStream_t stream) {
  if (nq == 0) return SSH_OK;
  const size_t need = rerank_workspace_bytes(nq, C);
  if ((int64_t)nq * C > INT32_MAX || need > kNoAllocScratch)
    return fail(SSH_ECAPACITY, "dtw_rerank_noalloc: nq * C = " + std::to_string((int64_t)nq * C) +
                                   " pairs need " + std::to_string(need) +
                                   " bytes of scratch, above SSH_NOALLOC_SCRATCH_BYTES");
  void* ws = nullptr;
  const ssh_status st = scratch_address(&ws);
  if (st != SSH_OK) return st;
  return rerank_launch(q, q_off, nq, db, db_off, Ndb, cand, ncand, C, band_frac, k, out_id,
                       out_dist, ws, kNoAllocScratch, stream);
}

}  // namespace ssh
