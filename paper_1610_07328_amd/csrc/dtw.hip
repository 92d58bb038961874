// Banded DTW re-rank (Section 2.1; the top-k step closing Algorithm 2).
//
// D(i,j) = (q_i - x_j)^2 + min(D(i-1,j), D(i,j-1), D(i-1,j-1)), D(0,0) = cost,
// cells with |i - j| > r or outside the matrix at +inf; distance = sqrt(D(lq-1, lx-1)).
//
// Layout: one (query, candidate) pair per 16-lane DPP row, four pairs per
// wavefront.  Lane L of a row owns G consecutive band offsets
// o = j - i = -r + L*G + g (g = 0..G-1) and walks the query rows, lane L
// handling row i = T - L at step T (a skew of one row per lane).  Within a
// lane the G cells of a row are computed left to right, each from its left
// neighbour (just computed), the cell above (the same lane's previous row at
// offset o+1) and the diagonal (previous row, same offset).  The two values a
// lane needs from its neighbours travel by DPP row shifts: the left of slot 0
// from lane L-1 (which finished row i one step earlier) and the upper cell of
// slot G-1 from lane L+1 (whose slot 0 of row i-1 is computed first in this
// step).  Row ends yield +inf through the DPP bound, which is the band edge
// (-r-1) on the left; on the right the first offset past the band (r+1) is
// held at +inf.  The x values of a lane's G cells shift by one slot per row,
// so a lane loads one new x per row; in the steady state the ring of x
// registers is renamed by unrolling G rows instead of moved.
//
// Each cell costs one subtract, one three-way min, one fused multiply-add and
// one add of a per-slot constant in float32: the constant is +inf for the one
// slot that holds the first offset past the band (offset r + 1) and 0 for every
// other slot, which keeps that slot at +inf without a select (all cell values
// are >= 0, so adding 0 is exact).  In the steady state, blocks of rows whose
// x indices are provably inside the series on every lane load x unchecked,
// and each block's q and x values are loaded one block ahead.
//
// The kernel computes either every (query, column) pair or the pairs a slot
// list names; the LB_Keogh-pruned re-rank at the end of this file uses two
// such lists (the best-bound candidates, then the survivors).
#include <cmath>

#include "common.hpp"

namespace ssh {

constexpr float kInf = __builtin_inff();
constexpr int kSegLanes = 16;
constexpr int kPrologue = kSegLanes - 1;

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

struct DtwLane {
  const float* qs;  // query values
  const float* xs;  // candidate values
  int lq, lx;
  int L;            // lane in its row
  int jn;           // x index of slot G-1 for the next row
  bool clampLane;   // holds the first offset past the band
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

template <int G>
__global__ __launch_bounds__(256) void dtw_kernel(const float* __restrict__ q,
                                                  const int64_t* __restrict__ q_off, int nq,
                                                  const float* __restrict__ db,
                                                  const int64_t* __restrict__ db_off, int64_t Ndb,
                                                  const int64_t* __restrict__ cand,
                                                  const int32_t* __restrict__ ncand, int C, int lq,
                                                  int lx, int r, float* __restrict__ dist, int* err,
                                                  const int32_t* __restrict__ plist, int64_t nslots) {
  static_assert(G >= 2, "at least two offsets per lane");
  const int lane = lane_id();
  const int L = lane & (kSegLanes - 1);
  const int64_t slot = ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * 4 + (lane >> 4);
  const int64_t npairs = (int64_t)nq * C;
  // with a slot list, slot i computes pair plist[i] (-1: none) and writes only
  // that pair's distance; without one, slot i is pair i
  int64_t pair = slot;
  if (plist != nullptr) pair = slot < nslots ? plist[slot] : -1;
  const bool inb = plist != nullptr ? pair >= 0 : pair < npairs;
  const int64_t qi = inb ? pair / C : nq - 1;
  const int ci = inb ? (int)(pair - qi * C) : 0;
  bool live = inb && ci < ncand[qi];
  const bool writes = plist == nullptr ? inb : live;
  int64_t id = 0;
  if (live) {
    id = cand[pair];
    if (id < 0 || id >= Ndb || db_off[id + 1] - db_off[id] != lx ||
        q_off[qi + 1] - q_off[qi] != lq) {
      if (L == 0) atomicOr(err, 1);
      live = false;
    }
  }
  if (ballot64(live) == 0) {
    if (writes && L == 0) dist[pair] = kInf;
    return;
  }
  // A lane without a pair borrows the query of the first live lane of its
  // wave (whose length was checked to be lq) for both its q and x reads.
  const int src = __builtin_ctzll(ballot64(live));
  const int64_t qsel = __shfl(live ? qi : (int64_t)0, src, kWave);
  DtwLane d;
  d.qs = q + q_off[live ? qi : qsel];
  d.xs = live ? db + db_off[id] : d.qs;
  d.lq = lq;
  d.lx = live ? lx : lq;
  d.L = L;
  const int span = 2 * r + 1;  // first offset past the band: -r + span
  const int Lv = span / G, gv = span % G;
  d.clampLane = L == Lv;
  const int L0 = r / G, g0 = r % G;  // slot of offset 0 (holds D(-1,-1) = 0)
  // the first offset past the band (slot gv of lane Lv) stays +inf: its cost
  // gets +inf added; every other cell adds 0 (exact: all values are >= 0)
  float cb[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cb[g] = (d.clampLane && g == gv) ? kInf : 0.0f;
  // At step T lane L is on row i = T - L; its x ring holds x[i + o] for its G
  // offsets o, so at T = 0 (row -L) it starts at x[L(G-1) - r + g].
  float V[G], xr[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    V[g] = (L == L0 && g == g0) ? 0.0f : kInf;
    xr[g] = x_at(d, L * (G - 1) - r + g);
  }
  d.jn = L * (G - 1) - r + G;  // slot G-1 of row -L + 1
  const int Ttot = lq + kPrologue;
  int T = 0;
  const int p_end = kPrologue < lq ? kPrologue : lq;
  for (; T < p_end; ++T) step_masked<G>(d, V, xr, T, cb);
  if (T == kPrologue) {
    const int full = (lq - kPrologue) / G * G;
    const int T_end = kPrologue + full;
    // At step T lane L loads x[T + L(G-1) - r + G].  Over a block of G steps
    // from T0 the indices span [T0 - r + G, T0 + 17G - 16 - r] (lanes 0 and
    // 15), inside [0, min(lx, lq)) -- every lane's x, a borrowed query of
    // length lq included, is that long -- when T0 >= r - G and
    // T0 <= min(lx, lq) + 15 - 17G + r.
    const int lmin = lx < lq ? lx : lq;
    const int in_lo = r - G;
    const int in_hi = lmin + (kSegLanes - 1) - (kSegLanes + 1) * G + r;  // last T0 allowed
    // each block's loads are issued one block ahead, while the previous block
    // computes
    // two buffers in turn, so that no values are copied between blocks
    float qa[G], xa[G], qc[G], xc[G];
    auto in_at = [&](int T0) { return T0 >= in_lo && T0 <= in_hi; };
    if (kPrologue < T_end) load_block<G>(d, kPrologue, d.jn, in_at(kPrologue), qa, xa);
    for (int T0 = kPrologue; T0 < T_end; T0 += 2 * G) {
      const int T1 = T0 + G, T2 = T0 + 2 * G;
      if (T1 < T_end) load_block<G>(d, T1, d.jn + G, in_at(T1), qc, xc);
      steps_full<G, 0>(d, V, xr, qa, xa, cb);
      if (T1 >= T_end) break;
      if (T2 < T_end) load_block<G>(d, T2, d.jn + G, in_at(T2), qa, xa);
      steps_full<G, 0>(d, V, xr, qc, xc, cb);
    }
    T = T_end;
  }
  for (; T < Ttot; ++T) step_masked<G>(d, V, xr, T, cb);

  // D(lq-1, lx-1) sits at offset lx - lq
  const int of = lx - lq;
  if (writes) {
    float res = kInf;
    if (of >= -r && of <= r) {
      const int Lf = (of + r) / G, gf = (of + r) % G;
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (g == gf) res = V[g];
      if (L == Lf) dist[pair] = live ? __builtin_sqrtf(res) : kInf;
    } else if (L == 0) {
      dist[pair] = kInf;
    }
  }
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
// LB_Keogh pruning (the lower-bound step before exact DTW; Section 2.1 and the
// pruning the paper's re-rank relies on).  For candidate value x_j the query
// values it can be matched with are q_i, |i - j| <= r, so every warping path
// pays at least the squared distance from x_j to [min, max] of that window:
//     LB = sum_j dist(x_j, [Lo_j, U_j])^2 <= D (the DTW total cost).
// A query's k candidates with the smallest LB are computed first; the largest
// of their distances, tau, bounds the k-th best, and a candidate is skipped
// when its LB exceeds tau^2 by more than every rounding involved can account
// for (the factor passed as prune_f, see rerank_lb_launch), which leaves its
// distance strictly above the k-th best: the top k are those of dtw_rerank.
// ---------------------------------------------------------------------------

constexpr int kLbLds = 4096;   // envelope values staged in LDS for the bounds

// Envelope of each query over the candidate index j in [0, lx): the window
// q[max(0, j - r), min(lq - 1, j + r)].  One workgroup per query and 256
// consecutive j, with the query values their windows cover (at most 256 +
// 2 SSH_MAX_BAND) staged in LDS.  An empty window (no alignment for x_j) gets
// U = -inf, Lo = +inf.  A query whose length is not lq gets the widest
// envelope (LB = 0: never skipped; the DTW step reports the length).
constexpr int kEnvJ = 256;
__global__ __launch_bounds__(kEnvJ) void lb_envelope_kernel(const float* __restrict__ q,
                                                            const int64_t* __restrict__ q_off,
                                                            int lq, int lx, int r,
                                                            float* __restrict__ U,
                                                            float* __restrict__ Lo) {
  __shared__ float qsh[kEnvJ + 2 * SSH_MAX_BAND + 1];
  const int jblocks = (lx + kEnvJ - 1) / kEnvJ;
  const int qi = blockIdx.x / jblocks;
  const int j0 = (blockIdx.x - qi * jblocks) * kEnvJ;
  const bool ok = q_off[qi + 1] - q_off[qi] == lq;
  const float* qs = q + q_off[qi];
  const int s0 = j0 - r < 0 ? 0 : j0 - r;
  const int s1 = j0 + kEnvJ + r < lq ? j0 + kEnvJ + r : lq;  // staged q[s0, s1)
  if (ok)
    for (int i = s0 + (int)threadIdx.x; i < s1; i += kEnvJ) qsh[i - s0] = qs[i];
  __syncthreads();
  const int j = j0 + (int)threadIdx.x;
  if (j >= lx) return;
  float mx = -kInf, mn = kInf;
  if (ok) {
    const int a = j - r < 0 ? 0 : j - r;
    const int b = j + r < lq - 1 ? j + r : lq - 1;
    for (int i = a; i <= b; ++i) {
      const float v = qsh[i - s0];
      mx = fmaxf(mx, v);
      mn = fminf(mn, v);
    }
  } else {
    mx = kInf;
    mn = -kInf;
  }
  U[(int64_t)qi * lx + j] = mx;
  Lo[(int64_t)qi * lx + j] = mn;
}

// LB_Keogh of every live pair (float32 sum): one workgroup per query and four
// of its candidates, one wavefront each, the query's envelope in LDS when
// lx <= kLbLds.  An invalid candidate (id or length) gets 0 and is left to the
// DTW step.
__global__ __launch_bounds__(256) void lb_keogh_kernel(const float* __restrict__ db,
                                                       const int64_t* __restrict__ db_off,
                                                       int64_t Ndb, const int64_t* __restrict__ cand,
                                                       const int32_t* __restrict__ ncand, int C,
                                                       int lx, const float* __restrict__ U,
                                                       const float* __restrict__ Lo,
                                                       float* __restrict__ lb) {
  extern __shared__ float env[];  // U then Lo, lx each, when staged
  const int groups = (C + 3) / 4;
  const int qi = blockIdx.x / groups;
  const int c0 = (blockIdx.x - qi * groups) * 4;
  const int nc = ncand[qi] < C ? ncand[qi] : C;
  if (c0 >= nc) return;  // no candidate here (uniform over the workgroup)
  const bool staged = lx <= kLbLds;
  const float* u = U + (int64_t)qi * lx;
  const float* lo = Lo + (int64_t)qi * lx;
  if (staged) {
    for (int j = threadIdx.x; j < lx; j += blockDim.x) {
      env[j] = u[j];
      env[lx + j] = lo[j];
    }
    u = env;
    lo = env + lx;
  }
  __syncthreads();
  const int ci = c0 + threadIdx.x / kWave;
  if (ci < nc) {
    const int64_t pair = (int64_t)qi * C + ci;
    const int64_t id = cand[pair];
    const bool ok = id >= 0 && id < Ndb && db_off[id + 1] - db_off[id] == lx;
    float s = 0.0f;
    if (ok) {
      const float* xs = db + db_off[id];
      for (int j = lane_id(); j < lx; j += kWave) {
        const float x = xs[j];
        const float t = x > u[j] ? x - u[j] : (x < lo[j] ? lo[j] - x : 0.0f);
        s = __builtin_fmaf(t, t, s);
      }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (lane_id() == 0) lb[pair] = s;
  }
}

// Per query: distances preset to +inf; the k live candidates with the
// smallest LB (ties by column) marked 1 and listed in the first pass's slots
// list1[qi k ..) (-1 past the live count), the other live candidates marked 2,
// the rest 0.
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

// Per query, after the first pass: tau = the largest first-pass distance;
// the candidates marked 2 whose LB does not exceed tau^2 prune_f fill the
// second pass's slots list2[qi (C - k) ..), the rest of which get -1 (a
// dropped candidate keeps its +inf distance).
__global__ __launch_bounds__(256) void lb_prune_kernel(const float* __restrict__ lb,
                                                       const float* __restrict__ dist,
                                                       const int32_t* __restrict__ ncand, int C,
                                                       int k, float prune_f,
                                                       const uint8_t* __restrict__ mark,
                                                       int32_t* __restrict__ list2) {
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
  const float cut = tau * tau * prune_f;  // +inf when tau is +inf: nothing is dropped
  int32_t* l2 = list2 + (int64_t)qi * (C - k);
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int64_t p = (int64_t)qi * C + i;
    if (mark[p] == 2 && !(lb[p] > cut)) l2[atomicAdd(&nkeep, 1u)] = (int32_t)p;
  }
  __syncthreads();
  for (int i = (int)nkeep + threadIdx.x; i < C - k; i += blockDim.x) l2[i] = -1;
}

__device__ int g_dtw_err;

int take_dtw_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_dtw_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_dtw_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

size_t rerank_workspace_bytes(int nq, int C) { return ((size_t)nq * C * sizeof(float) + 255) & ~(size_t)255; }

template <int G>
static void launch_g(unsigned grid, hipStream_t s, const float* q, const int64_t* q_off, int nq,
                     const float* db, const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                     const int32_t* ncand, int C, int lq, int lx, int r, float* dist, int* err,
                     const int32_t* plist, int64_t nslots) {
  dtw_kernel<G><<<grid, 256, 0, s>>>(q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist,
                                      err, plist, nslots);
}

// The DTW kernel of the smallest lane width G that holds the band (16 G >=
// 2 r + 2), over every pair (plist null) or the nslots pairs plist lists.
static ssh_status launch_dtw(hipStream_t stream, const float* q, const int64_t* q_off, int nq,
                             const float* db, const int64_t* db_off, int64_t Ndb,
                             const int64_t* cand, const int32_t* ncand, int C, int lq, int lx,
                             int r, float* dist, int* err, const int32_t* plist, int64_t nslots) {
  const int64_t n = plist != nullptr ? nslots : (int64_t)nq * C;
  if (n == 0) return SSH_OK;
  const unsigned grid = (unsigned)ceil_div(n, 16);
  const int need = 2 * r + 2;  // band offsets plus the +inf guard offset
#define SSH_G(GG)                                                                                 \
  if (kSegLanes * GG >= need) {                                                                   \
    launch_g<GG>(grid, stream, q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist, err, \
                 plist, nslots);                                                                  \
  } else
  SSH_G(2) SSH_G(3) SSH_G(4) SSH_G(5) SSH_G(6) SSH_G(7) SSH_G(8) SSH_G(10) SSH_G(12) SSH_G(14)
  SSH_G(16) SSH_G(20) SSH_G(24) SSH_G(26) SSH_G(28) SSH_G(32) {
    return fail(SSH_EUNSUPPORTED, "dtw_rerank: band too wide");
  }
#undef SSH_G
  return check_launch("dtw_rerank");
}

ssh_status rerank_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                         const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                         const int32_t* ncand, int C, float band_frac, int64_t q_len,
                         int64_t db_len, int k, int64_t* out_id, float* out_dist, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  if (nq == 0) return SSH_OK;
  if (ws_bytes < rerank_workspace_bytes(nq, C)) return fail(SSH_EINVAL, "dtw_rerank: workspace too small");
  const int64_t mx = q_len > db_len ? q_len : db_len;
  const int r = (int)std::floor((double)band_frac * (double)mx);
  if (r > SSH_MAX_BAND) return fail(SSH_EUNSUPPORTED, "dtw_rerank: band radius above SSH_MAX_BAND");
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_dtw_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "dtw_rerank: cannot resolve error flag");
  float* dist = reinterpret_cast<float*>(ws);
  const int lq = (int)q_len, lx = (int)db_len;
  ssh_status st = launch_dtw(stream, q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r,
                             dist, err, nullptr, 0);
  if (st != SSH_OK) return st;
  topk_kernel<<<nq, 256, 0, stream>>>(dist, cand, ncand, C, k, out_id, out_dist);
  return check_launch("dtw_rerank");
}

// Workspace of the pruned re-rank: distances and LB [nq][C] (float32), marks
// [nq][C] (u8), the two passes' slot lists (nq k, then nq (C - k), int32),
// the query envelopes U and Lo [nq][lx] (float32).
static inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
size_t rerank_lb_workspace_bytes(int nq, int C, int64_t lx) {
  const size_t pc = (size_t)nq * C;
  return 3 * al256(pc * 4) + al256(pc) + 2 * al256((size_t)nq * lx * 4);
}

ssh_status rerank_lb_launch(const float* q, const int64_t* q_off, int nq, const float* db,
                            const int64_t* db_off, int64_t Ndb, const int64_t* cand,
                            const int32_t* ncand, int C, float band_frac, int64_t q_len,
                            int64_t db_len, int k, int64_t* out_id, float* out_dist, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  if (nq == 0) return SSH_OK;
  if (ws_bytes < rerank_lb_workspace_bytes(nq, C, db_len))
    return fail(SSH_EINVAL, "dtw_rerank_lb: workspace too small");
  if ((int64_t)nq * ((C + 3) / 4) > INT32_MAX || (int64_t)nq * ((db_len + 255) / 256) > INT32_MAX)
    return fail(SSH_EUNSUPPORTED, "dtw_rerank_lb: batch too large for one launch");
  const int64_t mx = q_len > db_len ? q_len : db_len;
  const int r = (int)std::floor((double)band_frac * (double)mx);
  if (r > SSH_MAX_BAND) return fail(SSH_EUNSUPPORTED, "dtw_rerank: band radius above SSH_MAX_BAND");
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_dtw_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "dtw_rerank: cannot resolve error flag");
  const int lq = (int)q_len, lx = (int)db_len;
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
  float* U = reinterpret_cast<float*>(p);
  p += al256((size_t)nq * lx * 4);
  float* Lo = reinterpret_cast<float*>(p);
  // Skip factor.  The float32 DTW total of a path of P <= lq + lx - 1 cells is
  // at least (1 - 2^-24)^(P + 2) times the exact one, the float32 LB at most
  // (1 + 2^-24)^(lx + 4) times the exact LB, and tau^2 recomputed from the
  // rounded square root is within 9 ulps of the total it came from; twice
  // their sum, plus 2^-19 so that the rounded distances differ strictly.
  const double m = (double)(q_len + 2 * db_len + 64) * 0x1p-23 + 0x1p-19;
  float prune_f = (float)(1.0 + m);
  if ((double)prune_f < 1.0 + m) prune_f = std::nextafter(prune_f, INFINITY);
  lb_envelope_kernel<<<(unsigned)((int64_t)nq * ((lx + kEnvJ - 1) / kEnvJ)), kEnvJ, 0, stream>>>(
      q, q_off, lq, lx, r, U, Lo);
  const size_t lb_lds = lx <= kLbLds ? (size_t)lx * 8 : 0;
  lb_keogh_kernel<<<(unsigned)((int64_t)nq * ((C + 3) / 4)), 256, lb_lds, stream>>>(
      db, db_off, Ndb, cand, ncand, C, lx, U, Lo, lb);
  lb_select_kernel<<<nq, 256, 0, stream>>>(lb, ncand, C, k, mark, dist, list1);
  ssh_status st = check_launch("dtw_rerank_lb");
  if (st != SSH_OK) return st;
  st = launch_dtw(stream, q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist, err,
                  list1, (int64_t)nq * k);
  if (st != SSH_OK) return st;
  if (C > k) {
    lb_prune_kernel<<<nq, 256, 0, stream>>>(lb, dist, ncand, C, k, prune_f, mark, list2);
    st = launch_dtw(stream, q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist, err,
                    list2, (int64_t)nq * (C - k));
    if (st != SSH_OK) return st;
  }
  topk_kernel<<<nq, 256, 0, stream>>>(dist, cand, ncand, C, k, out_id, out_dist);
  return check_launch("dtw_rerank_lb");
}

}  // namespace ssh
