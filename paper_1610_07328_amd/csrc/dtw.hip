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
// x indices are provably inside the series on every lane load x unchecked.
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
                                                  int lx, int r, float* __restrict__ dist, int* err) {
  static_assert(G >= 2, "at least two offsets per lane");
  const int lane = lane_id();
  const int L = lane & (kSegLanes - 1);
  const int64_t pair = ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * 4 + (lane >> 4);
  const int64_t npairs = (int64_t)nq * C;
  const int64_t qi = pair < npairs ? pair / C : nq - 1;
  const int ci = pair < npairs ? (int)(pair - qi * C) : 0;
  bool live = pair < npairs && ci < ncand[qi];
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
    if (pair < npairs && L == 0) dist[pair] = kInf;
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
  if (pair < npairs) {
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
                     const int32_t* ncand, int C, int lq, int lx, int r, float* dist, int* err) {
  dtw_kernel<G><<<grid, 256, 0, s>>>(q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist,
                                      err);
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
  const int64_t npairs = (int64_t)nq * C;
  const unsigned grid = (unsigned)ceil_div(npairs, 16);
  const int need = 2 * r + 2;  // band offsets plus the +inf guard offset
  const int lq = (int)q_len, lx = (int)db_len;
#define SSH_G(GG)                                                                                 \
  if (kSegLanes * GG >= need) {                                                                   \
    launch_g<GG>(grid, stream, q, q_off, nq, db, db_off, Ndb, cand, ncand, C, lq, lx, r, dist, err); \
  } else
  SSH_G(2) SSH_G(3) SSH_G(4) SSH_G(5) SSH_G(6) SSH_G(7) SSH_G(8) SSH_G(10) SSH_G(12) SSH_G(14)
  SSH_G(16) SSH_G(20) SSH_G(24) SSH_G(26) SSH_G(28) SSH_G(32) {
    return fail(SSH_EUNSUPPORTED, "dtw_rerank: band too wide");
  }
#undef SSH_G
  ssh_status st = check_launch("dtw_rerank");
  if (st != SSH_OK) return st;
  topk_kernel<<<nq, 256, 0, stream>>>(dist, cand, ncand, C, k, out_id, out_dist);
  return check_launch("dtw_rerank");
}

}  // namespace ssh
