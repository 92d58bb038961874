// Weighted MinHash of the shingle sets by consistent weighted sampling
// (Section 4.3, and Section 2, eqs. WJaccardDef / CollProb), following Ioffe's
// improved consistent weighted sampling, the sampler the paper cites.
//
// For hash j and token k of weight S (draws r ~ Gamma(2,1), ln c, beta ~ U[0,1)):
//     t    = floor(ln S / r + beta)
//     ln y = r (t - beta)
//     ln a = ln c - ln y - r
// k* = argmin_k ln a (ties to the smaller k), hv = min(t*, 2^47-1) << 16 | k*
// (at most 2^63 - 1, so no hash value equals the empty-series value 2^64 - 1).
// Every step is one correctly rounded float64 operation, in this order; the
// library is compiled without floating-point contraction so no step fuses.
// ln S comes from a table of correctly rounded logarithms prepared once on
// the device by a double-double evaluation (and is evaluated the same way on
// the fly for the rare count beyond the table).
//
// One wavefront hashes one series, each lane two hashes.  The exact argmin is
// found in two passes whose combination equals the first minimum of the
// ascending float64 scan, i.e. the lexicographic minimum of (ln a, k):
//  A. keyed tokens (all of them in practice): tokens of weight 1..31, and
//     the two run codes 0 and 2^n - 1 (which collect the constant stretches of
//     the bit stream and alone reach large weights) up to weight 4096.  The
//     prepare kernel stores, per (key row, hash), a 16-bit key that is a
//     monotone (non-decreasing) quantisation of the exact ln a.  A strictly
//     smaller key therefore means a strictly smaller ln a.  Each lane keeps
//     the smallest and second-smallest (key << 16 | position); position order
//     is token order, so equal keys resolve to the earlier token.  If the
//     smallest key is shared by two tokens (rare), the lane evaluates exactly
//     the keyed tokens holding that key.
//  B. any other token (heavy): pass A lists up to 64 of them in LDS with
//     their ln S (beyond that, pass B relists them one chunk at a time); every
//     lane evaluates each of them exactly for its two hashes and compares by
//     (ln a, k) with the pass-A winner, whose ln a is then evaluated exactly.
// Batches of fewer than kSplitN series give each series a whole workgroup:
// its four waves run pass A over alternate blocks of tokens and merge their
// two smallest composites per hash, and the first wave finishes the series.
// With band keys requested, the kernel also folds each series' hash values
// into its L band keys (Algorithm 1) from a copy it keeps in LDS.
#include <algorithm>
#include <cmath>

#include "band.hpp"

namespace ssh {

// ---------------------------------------------------------------------------
// double-double arithmetic (error-free transforms; needs no contraction)
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return {p, e};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
  double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}

// ln(s) for an integer 1 <= s < 2^53, rounded to the nearest float64.
// s = 2^e f with f in (sqrt(2)/2, sqrt(2)]; ln f = 2 atanh((f-1)/(f+1)) summed
// in double-double to ~2^-100 relative, then e ln 2 added (ln 2 as a
// double-double constant).
__device__ double ln_integer(double s) {
  if (s == 1.0) return 0.0;
  const dd LN2 = {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56};
  int e = 0;
  double f = __builtin_frexp(s, &e);  // s = f 2^e, f in [0.5, 1)
  f *= 2.0;
  e -= 1;  // f in [1, 2)
  if (f > 1.4142135623730951) {
    f *= 0.5;
    e += 1;
  }
  const double num = f - 1.0;  // exact (Sterbenz)
  const dd den = two_sum(f, 1.0);
  const dd z = dd_div(dd{num, 0.0}, den);
  const dd z2 = dd_mul(z, z);
  dd term = z, sum = z;
  for (int k = 1; k <= 26; ++k) {
    term = dd_mul(term, z2);
    sum = dd_add(sum, dd_div(term, dd{(double)(2 * k + 1), 0.0}));
  }
  sum.hi *= 2.0;
  sum.lo *= 2.0;
  dd el = two_prod((double)e, LN2.hi);
  el.lo += (double)e * LN2.lo;
  el = fast_two_sum(el.hi, el.lo);
  const dd res = dd_add(el, sum);
  return res.hi + res.lo;
}

// the sampler's exact steps for a token of weight with log ls
__device__ __forceinline__ double icws_ln_a(double rr, double bb, double lc, double ls, double& tt) {
  tt = __builtin_floor(ls / rr + bb);
  const double ln_y = rr * (tt - bb);
  return (lc - ln_y) - rr;
}

__device__ __forceinline__ double lnS_of(const double* lnS, uint32_t c) {
  return c < (uint32_t)SSH_LNS_ENTRIES ? lnS[c] : ln_integer((double)c);
}

// ---------------------------------------------------------------------------
// prepare: lnS table, the weight-1 ln a of every (k, j), and the 16-bit keys
// ---------------------------------------------------------------------------
// Monotone non-decreasing 16-bit key of ln a.  For a token of weight S,
// a ~ Exp(S), so ln a < -16 has probability about S * 1.1e-7; such values
// saturate at key 0 and values above 4 at the top key (saturation only costs
// exact tie checks).  Keys stop at 0xFFFE so that no key equals the
// empty-minimum sentinel.
constexpr double kKeyLo = -16.0;
constexpr double kKeyScale = 65534.0 / 20.0;

constexpr uint32_t kKeyW = SSH_CWS_KEY_WEIGHTS;  // weights keyed for every code
constexpr uint32_t kRunCap = SSH_CWS_RUN_CAP;    // counts keyed for the two run codes
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

// Rows of the key table: weight w (1..kKeyW) of code k at (w - 1) 2^n + k;
// count c (1..kRunCap) of code 0 at kKeyW 2^n + c - 1 and of code 2^n - 1
// (the tokens of constant runs in the bit stream, the only ones that reach
// large weights) at kKeyW 2^n + kRunCap + c - 1; then one padding row.
__host__ __device__ inline int64_t key_rows(int n) {
  return ((int64_t)kKeyW << n) + 2 * (int64_t)kRunCap + 1;
}

// row of token (code, count c) or kNoRow when it is not keyed (c == 0 included)
__device__ __forceinline__ uint32_t key_row(uint32_t code, uint32_t c, int n) {
  if (c - 1u < kKeyW) return ((c - 1u) << n) + code;
  if (c <= kRunCap && (code == 0u || code == (1u << n) - 1u))
    return (kKeyW << n) + (code ? kRunCap : 0u) + c - 1u;
  return kNoRow;
}

// The key table is stored in column chunks of kKeyChunk hashes, chunk-major:
// chunk q holds the keys of hashes 128 q .. 128 q + c_q - 1 of every row, row
// after row, at a row width w_q of c_q rounded up to even, or of 128 where c_q
// is above 96: one pass of 128 hashes then reads whole, contiguous row
// segments, and a row of 97 to 128 hashes starts on a 256-byte boundary
// (2 cache lines per token, where a 200-byte stride averages 2.6).
constexpr int kKeyChunk = 128;
static_assert(kKeyChunk == 2 * kWave, "one pass of the main kernel covers one key chunk");
__host__ __device__ inline int key_chunk_width(int H, int q) {
  int w = H - kKeyChunk * q < kKeyChunk ? H - kKeyChunk * q : kKeyChunk;
  w += w & 1;
  return w > 96 ? kKeyChunk : w;
}
__host__ __device__ inline int key_table_cols(int H) {
  const int nq = (H + kKeyChunk - 1) / kKeyChunk;
  return kKeyChunk * (nq - 1) + key_chunk_width(H, nq - 1);
}

__device__ __forceinline__ uint32_t key16(double la) {
  const double q = __builtin_floor((la - kKeyLo) * kKeyScale);  // monotone steps
  const double c = q < 0.0 ? 0.0 : (q > 65534.0 ? 65534.0 : q);
  return (uint32_t)c;
}

// the lnS table: correctly rounded ln s for every s < SSH_LNS_ENTRIES
__global__ __launch_bounds__(256) void cws_lns_kernel(double* __restrict__ lnS) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < SSH_LNS_ENTRIES; s += stride)
    lnS[s] = s == 0 ? -INFINITY : ln_integer((double)s);
}

// the key rows, the weight-1 ln a and the (r, beta) table; ln w from the lnS
// table written by cws_lns_kernel before it on the stream
__global__ __launch_bounds__(256) void cws_prepare_kernel(
    const double* __restrict__ r, const double* __restrict__ lnc, const double* __restrict__ beta,
    int n, int H, double* __restrict__ a1, uint16_t* __restrict__ k16,
    const double* __restrict__ lnS, double2* __restrict__ rb, int* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t rows = key_rows(n);
  const int64_t cells = rows * key_table_cols(H);
  const uint32_t wrows = kKeyW << n;  // rows of the per-weight part
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += stride) {
    // chunk q starts at element rows * 128 q; row and column inside it
    const int q = (int)(c / (rows * kKeyChunk));
    const int wq = key_chunk_width(H, q);
    const int64_t e = c - rows * kKeyChunk * q;
    const int64_t row = e / wq;
    const int j = kKeyChunk * q + (int)(e - row * wq);
    if (j >= H || row == rows - 1) {  // padding column or row, never wins a minimum
      k16[c] = 0xFFFF;
      continue;
    }
    uint32_t code, w;
    if (row < wrows) {
      code = (uint32_t)row & ((1u << n) - 1u);
      w = (uint32_t)(row >> n) + 1u;
    } else {
      const uint32_t q = (uint32_t)(row - wrows);
      code = q < kRunCap ? 0u : (1u << n) - 1u;
      w = q % kRunCap + 1u;
    }
    const int64_t i = (int64_t)code * H + j;
    const double rr = r[i], bb = beta[i], lc = lnc[i];
    const double ls = lnS[w];  // the table's correctly rounded ln w (w <= SSH_CWS_RUN_CAP)
    double tt;
    const double a = icws_ln_a(rr, bb, lc, ls, tt);
    k16[c] = (uint16_t)key16(a);
    if (row < (1 << n)) {  // weight 1: the ln a and (r, beta) tables, range checks of the draws
      a1[i] = a;
      rb[i] = make_double2(rr, bb);
      // r is bounded so that the float64 rounding of ln a stays far below the
      // pass-B slack (a Gamma(2,1) draw above 1e5 has probability ~e^-1e5)
      if (!(rr > 0.0) || !(rr < 1.0e5) || !(bb >= 0.0) || !(bb < 1.0) ||
          !(__builtin_fabs(lc) < 1.0e300))
        atomicOr(err, 2);
    }
  }
}

// ---------------------------------------------------------------------------
// main
// ---------------------------------------------------------------------------
struct CwsDev {
  const double* lnc;
  const double* a1;
  const double* lnS;
  const uint16_t* k16;  // key_rows(n) rows in column chunks; the last row is padding
  const double2* rb;    // [2^n][H] (r, beta)
  int H, n;
};

constexpr int kCwsWaves = 4;  // wavefronts per workgroup
constexpr int kPassA = 16;     // keyed tokens whose keys are loaded together
constexpr int kHeavyCap = 64; // heavy tokens listed per series in LDS
constexpr int kBandLds = 256; // hash values kept per wave in LDS for the fused band keys
constexpr int64_t kSplitN = 4096;  // below this many series, a workgroup per series
constexpr uint32_t kNone = 0xFFFFFFFFu;

// median of three; with a <= b it is the second smallest of {a, b, c}
__device__ __forceinline__ uint32_t med3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t m;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(m) : "v"(a), "v"(b), "v"(c));
  return m;
}

__device__ __forceinline__ double exact_ln_a(const CwsDev& t, uint32_t k, uint32_t c, int j,
                                             double& tt) {
  const int64_t i = (int64_t)k * t.H + j;
  if (c == 1u) {
    tt = 0.0;
    return t.a1[i];
  }
  const double2 q = t.rb[i];
  return icws_ln_a(q.x, q.y, t.lnc[i], lnS_of(t.lnS, c), tt);
}

struct Best {
  double la;  // exact ln a of the minimum (+inf if none)
  uint32_t k;
  double t;
};

// Band keys computed by the CWS kernel from the hash values it holds (H = K L,
// H <= kBandLds): the same fold as the band-key kernel.  A wave keeps the hash
// values of G consecutive series of its own in LDS and folds their G L bands
// at once, one band per lane.
struct BandOut {
  uint64_t* keys;  // [N][L]
  int K, L;
  uint64_t seed;
  int G;  // series per fold: min(64 / L, kBandLds / H), at least 1
};

// SPLIT (small batches): the four waves of a workgroup share one series.  Each
// runs pass A over every fourth block of 64 tokens; their two smallest
// composites per hash are merged through LDS (positions are the series' own,
// so the merged pair is the pair pass A over all tokens gives), and wave 0
// finishes the series: ties, pass B over the four heavy lists, output, keys.
template <bool KEYS, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void cws_kernel(
    const uint32_t* __restrict__ codes, const uint32_t* __restrict__ counts,
    const int64_t* __restrict__ hist_off, const int32_t* __restrict__ n_distinct, int64_t N,
    CwsDev t, uint64_t* __restrict__ hv, int* err, BandOut bo) {
  // per wave: keyed-token list (row byte offset, position), padded to whole
  // groups with the padding row, and the heavy-token list (position)
  __shared__ uint4 klist[kCwsWaves][kWave / 2];
  // heavy tokens of the series: (code, count, ln count as two words)
  __shared__ uint4 hl[kCwsWaves][kHeavyCap];
  // hash values of the last G series, for the band keys
  __shared__ uint64_t hvs[kCwsWaves][KEYS ? kBandLds : 1];
  // SPLIT: each wave's (m1, m2) of its two hashes, heavy-token count and flag
  __shared__ uint4 mm[SPLIT ? kCwsWaves : 1][SPLIT ? kWave : 1];
  __shared__ int hn[kCwsWaves], ha[kCwsWaves];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int lane = lane_id();
  const int H = t.H;
  const uint32_t krows = (uint32_t)key_rows(t.n);  // the table is below 2^31 bytes
  uint2* klist2 = reinterpret_cast<uint2*>(klist[w]);
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const int64_t stride = SPLIT ? (int64_t)gridDim.x : (int64_t)gridDim.x * kCwsWaves;
  const bool lead = !SPLIT || w == 0;  // the wave that finishes a series
  int slot = 0;  // series held in hvs since the last fold
  // after series s: fold the held series once G are held or s is the wave's last
  auto band_step = [&](int64_t s) {
    if constexpr (KEYS) {
      if (++slot < bo.G && s + stride < N) return;
      wave_sync_lds();
      for (int i = lane; i < slot * bo.L; i += kWave) {
        const int g = i / bo.L, l = i - g * bo.L;
        const uint64_t* hr = &hvs[w][g * H];
        const int64_t sg = s - (int64_t)(slot - 1 - g) * stride;
        bo.keys[sg * bo.L + l] =
            hr[0] == SSH_HV_EMPTY ? SSH_KEY_EMPTY : band_fold(hr + l * bo.K, bo.K, l, bo.seed);
      }
      wave_sync_lds();
      slot = 0;
    }
  };
  for (int64_t s = SPLIT ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * kCwsWaves + w; s < N;
       s += stride) {
    const int D = n_distinct[s];
    uint64_t* out = hv + s * H;
    uint64_t* held = KEYS ? &hvs[w][slot * H] : nullptr;
    if (D <= 0) {
      if (lead) {
        for (int j = lane; j < H; j += kWave) out[j] = SSH_HV_EMPTY;
        if constexpr (KEYS)
          if (lane == 0) held[0] = SSH_HV_EMPTY;  // the fold tests the first value only
        band_step(s);
      }
      continue;
    }
    const int64_t ho = hist_off[s];
    const uint32_t* codes_s = codes + ho;
    const uint32_t* counts_s = counts + ho;
    for (int hb0 = 0; hb0 < H; hb0 += 2 * kWave) {
      const int j0 = hb0 + 2 * lane, j1 = j0 + 1;
      const bool v0 = j0 < H, v1 = j1 < H;
      // this pass's key chunk: its first key, row stride and padding row (bytes),
      // read through a bounds-checked view of the chunk (a lane past H reads
      // inside it)
      const int qk = hb0 / kKeyChunk;
      const uint32_t row_bytes = (uint32_t)key_chunk_width(H, qk) * 2u;
      const uint16_t* kchunk = t.k16 + (size_t)krows * (size_t)(kKeyChunk * qk);
      const uint32_t pad_row = (krows - 1u) * row_bytes;
      const __amdgpu_buffer_rsrc_t ktab = __builtin_amdgcn_make_buffer_rsrc(
          (void*)kchunk, 0, (int)(krows * row_bytes), 0x00020000);
      const uint32_t colb = (uint32_t)(v0 ? j0 - hb0 : 0) * 2u;  // byte offset in the row
      Best b[2] = {Best{INFINITY, 0u, 0.0}, Best{INFINITY, 0u, 0.0}};
      bool done[2] = {!v0, !v1};
      bool any_heavy = false;
      if (D <= 0xFFFF) {
        // ---- pass A over keyed tokens; the others (heavy) are listed ----
        uint32_t m1[2] = {kNone, kNone}, m2[2] = {kNone, kNone};
        int nhl = 0;  // heavy tokens seen; listed while nhl <= kHeavyCap
        for (int d0 = SPLIT ? w * kWave : 0; d0 < D; d0 += (SPLIT ? kCwsWaves : 1) * kWave) {
          const int nc = D - d0 < kWave ? D - d0 : kWave;
          const bool have = lane < nc;
          const uint32_t mcode = have ? codes_s[d0 + lane] : 0u;
          const uint32_t mcnt = have ? counts_s[d0 + lane] : 0u;
          const uint32_t row = have ? key_row(mcode, mcnt, t.n) : kNoRow;
          const bool keyed = row != kNoRow;
          const uint64_t km = ballot64(keyed);
          const bool heavy = have && !keyed;
          const uint64_t hmk = ballot64(heavy);
          if (heavy && nhl + (int)__builtin_popcountll(hmk) <= kHeavyCap) {
            const double ls = lnS_of(t.lnS, mcnt);
            const uint64_t lb = __builtin_bit_cast(uint64_t, ls);
            hl[w][nhl + __builtin_popcountll(hmk & lt_mask)] =
                make_uint4(mcode, mcnt, (uint32_t)lb, (uint32_t)(lb >> 32));
          }
          nhl += __builtin_popcountll(hmk);
          any_heavy |= hmk != 0;
          const int nk = __builtin_popcountll(km);
          const int nkp = (nk + kPassA - 1) & ~(kPassA - 1);
          if (keyed) {
            klist2[__builtin_popcountll(km & lt_mask)] = make_uint2(row * row_bytes, (uint32_t)(d0 + lane));
          }
          // slots nk..nkp-1 are padding (keys 0xFFFF, position 0xFFFF: kNone);
          // lane i writes slot i whether or not it holds a keyed token itself
          if (lane >= nk && lane < nkp) klist2[lane] = make_uint2(pad_row, 0xFFFFu);
          wave_sync_lds();
          if (v0) for (int i0 = 0; i0 < nk; i0 += kPassA) {
            uint32_t wv[kPassA], pv[kPassA];
#pragma unroll
            for (int u = 0; u < kPassA; u += 2) {
              const uint4 e = klist[w][(i0 + u) >> 1];
              pv[u] = e.y;
              pv[u + 1] = e.w;
              wv[u] = __builtin_amdgcn_raw_buffer_load_b32(ktab, (int)(e.x + colb), 0, 0);
              wv[u + 1] = __builtin_amdgcn_raw_buffer_load_b32(ktab, (int)(e.z + colb), 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kPassA; ++u) {
              // (key << 16 | position) as byte selects of (key pair, position)
              const uint32_t c0 = __builtin_amdgcn_perm(wv[u], pv[u], 0x05040100u);
              const uint32_t c1 = __builtin_amdgcn_perm(wv[u], pv[u], 0x07060100u);
              m2[0] = med3(m1[0], m2[0], c0);  // second smallest (m1 <= m2)
              m1[0] = c0 < m1[0] ? c0 : m1[0];
              m2[1] = med3(m1[1], m2[1], c1);
              m1[1] = c1 < m1[1] ? c1 : m1[1];
            }
          }
          wave_sync_lds();
        }
        if constexpr (SPLIT) {
          // the two smallest of two sorted pairs (m1 <= m2, o1 <= o2) are
          // min(m1, o1) and med3(m1, o1, min(m2, o2))
          mm[w][lane] = make_uint4(m1[0], m2[0], m1[1], m2[1]);
          if (lane == 0) {
            hn[w] = nhl;
            ha[w] = any_heavy ? 1 : 0;
          }
          __syncthreads();
          if (lead) {
            for (int ww = 1; ww < kCwsWaves; ++ww) {
              const uint4 o = mm[ww][lane];
              m2[0] = med3(m1[0], o.x, m2[0] < o.y ? m2[0] : o.y);
              m1[0] = o.x < m1[0] ? o.x : m1[0];
              m2[1] = med3(m1[1], o.z, m2[1] < o.w ? m2[1] : o.w);
              m1[1] = o.z < m1[1] ? o.z : m1[1];
              any_heavy |= ha[ww] != 0;
            }
          }
        }
        if (lead) {
        // winner of pass A, unless its key is shared (then: exact re-scan)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (done[h] || m1[h] == kNone) continue;
          if (((m1[h] ^ m2[h]) >> 16) == 0) continue;  // tie: resolved below
          const uint32_t p = m1[h] & 0xFFFFu;
          if (p >= (uint32_t)D) {  // cannot happen: every list entry read is a token or padding
            atomicOr(err, 4);
            done[h] = true;
            continue;
          }
          b[h].k = codes_s[p];
          if (any_heavy) b[h].la = exact_ln_a(t, b[h].k, counts_s[p], h ? j1 : j0, b[h].t);
          else {
            const uint32_t c = counts_s[p];
            b[h].la = 0.0;  // not needed: no pass B
            b[h].t = 0.0;
            if (c > 1u) {
              const int64_t i = (int64_t)b[h].k * H + (h ? j1 : j0);
              const double2 q = t.rb[i];  // one 16-byte read
              b[h].t = __builtin_floor(lnS_of(t.lnS, c) / q.x + q.y);
            }
          }
          if (!any_heavy) done[h] = true;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool tie = !done[h] && m1[h] != kNone && ((m1[h] ^ m2[h]) >> 16) == 0;
          if (tie) {
            // The keyed minimum is among the keyed tokens whose key equals the
            // smallest key K (a smaller key means a smaller ln a): evaluate
            // exactly those, ascending, strict <.  Heavy tokens follow below.
            const int j = h ? j1 : j0;
            const uint32_t K = m1[h] >> 16;
            Best e{INFINITY, 0u, 0.0};
            for (int d = 0; d < D; ++d) {
              const uint32_t c = counts_s[d];
              const uint32_t k = codes_s[d];
              const uint32_t krow = key_row(k, c, t.n);
              if (krow == kNoRow ||
                  (uint32_t)kchunk[krow * (row_bytes >> 1) + (uint32_t)(j - hb0)] != K)
                continue;
              double tt;
              const double la = exact_ln_a(t, k, c, j, tt);
              if (la < e.la) e = Best{la, k, tt};
            }
            b[h] = e;
            done[h] = !any_heavy;
          }
        }
        // ---- pass B over tokens of weight >= 4 ----
        if (any_heavy) {
          // the list built in pass A when it holds every heavy token; else the
          // heavy tokens of one chunk at a time
          bool listed = nhl <= kHeavyCap;
          if constexpr (SPLIT)
            for (int ww = 0; ww < kCwsWaves; ++ww) listed = listed && hn[ww] <= kHeavyCap;
          // listed: one list (SPLIT: one per wave); else chunks of 64 tokens
          const int nit = listed ? (SPLIT ? kCwsWaves : 1) : D;
          for (int d0 = 0; d0 < nit; d0 += listed ? 1 : kWave) {
            const int li = SPLIT && listed ? d0 : w;  // the list read
            int cnt = SPLIT && listed ? hn[d0] : nhl;
            if (!listed) {
              const int nc = D - d0 < kWave ? D - d0 : kWave;
              const bool have = lane < nc;
              const uint32_t mcode = have ? codes_s[d0 + lane] : 0u;
              const uint32_t mcnt = have ? counts_s[d0 + lane] : 0u;
              const bool heavy = have && key_row(mcode, mcnt, t.n) == kNoRow;
              const uint64_t hm = ballot64(heavy);
              if (heavy) {
                const uint64_t lb = __builtin_bit_cast(uint64_t, lnS_of(t.lnS, mcnt));
                hl[w][__builtin_popcountll(hm & lt_mask)] =
                    make_uint4(mcode, mcnt, (uint32_t)lb, (uint32_t)(lb >> 32));
              }
              cnt = __builtin_popcountll(hm);
              wave_sync_lds();
            }
            for (int i = 0; i < cnt; ++i) {
              const uint4 e = hl[li][i];
              const uint32_t k = e.x;
              const double ls = __builtin_bit_cast(double, ((uint64_t)e.w << 32) | e.z);
              const int64_t row = (int64_t)k * H;
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                if (done[h]) continue;
                const int j = h ? j1 : j0;
                double tt;
                const double2 q = t.rb[row + j];
                const double la = icws_ln_a(q.x, q.y, t.lnc[row + j], ls, tt);
                if (la < b[h].la || (la == b[h].la && k < b[h].k)) b[h] = Best{la, k, tt};
              }
            }
            wave_sync_lds();
          }
        }
        }  // lead
      } else if (lead) {
        // more distinct tokens than 16-bit positions: plain exact scan
        for (int d = 0; d < D; ++d) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (done[h]) continue;
            double tt;
            const double la = exact_ln_a(t, codes_s[d], counts_s[d], h ? j1 : j0, tt);
            if (la < b[h].la) b[h] = Best{la, codes_s[d], tt};
          }
        }
      }
      const double tmax = 140737488355327.0;  // 2^47 - 1: hv stays below SSH_HV_EMPTY
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (lead && (h ? v1 : v0)) {
          const uint64_t tq = (uint64_t)(b[h].t < tmax ? b[h].t : tmax);
          const uint64_t v = (tq << 16) | (uint64_t)b[h].k;
          out[h ? j1 : j0] = v;
          if constexpr (KEYS) held[h ? j1 : j0] = v;
        }
      }
      if constexpr (SPLIT) __syncthreads();  // klist, hl and mm are reused next
    }
    if (lead) band_step(s);
  }
}

__device__ int g_cws_err;

int take_cws_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_cws_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_cws_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

int64_t cws_key_table_elems(int n, int H) {
  if (n < 1 || n > SSH_MAX_N || H < 1) return 0;
  return key_rows(n) * key_table_cols(H);
}

ssh_status cws_prepare_launch(const ssh_cws_tables* tab, hipStream_t stream) {
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_cws_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_cws_prepare: cannot resolve error flag");
  cws_lns_kernel<<<grid_for(SSH_LNS_ENTRIES, 256, 4096), 256, 0, stream>>>(tab->lnS);
  cws_prepare_kernel<<<grid_for(key_rows(tab->n) * key_table_cols(tab->H), 256, 4096), 256, 0,
                       stream>>>(
      tab->r, tab->lnc, tab->beta, tab->n, tab->H, tab->a1, tab->k16, tab->lnS,
      reinterpret_cast<double2*>(tab->rb), err);
  return check_launch("ssh_cws_prepare");
}

ssh_status band_keys_launch(const uint64_t* hv, int64_t N, int K, int L, uint64_t seed,
                            uint64_t* keys, hipStream_t stream);

// keys == nullptr: hash values only; else also the band keys of (K, L, seed),
// in the same kernel while H fits its LDS copy, else by the band-key kernel
ssh_status cws_launch(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                      const int32_t* n_distinct, int64_t N, const ssh_cws_tables* tab, uint64_t* hv,
                      uint64_t* keys, int K, int L, uint64_t seed, hipStream_t stream) {
  if (N == 0) return SSH_OK;
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_cws_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_cws: cannot resolve error flag");
  // the key table is addressed by 32-bit byte offsets through a buffer resource
  if (key_rows(tab->n) * key_table_cols(tab->H) * 2 >= (1ll << 31))
    return fail(SSH_EUNSUPPORTED, "ssh_cws: key table of 2 GiB or more");
  CwsDev t{tab->lnc, tab->a1, tab->lnS, tab->k16,
           reinterpret_cast<const double2*>(tab->rb), tab->H, tab->n};
  const unsigned grid = grid_for(N, kCwsWaves, 1 << 16);
  const bool fused = keys != nullptr && tab->H <= kBandLds;
  // small batches (one series per wave would leave most of the GPU idle): a
  // workgroup per series
  const bool split = N < kSplitN;
  const unsigned sgrid = grid_for(N, 1, 1 << 16);
  const BandOut bo = fused ? BandOut{keys, K, L, seed, std::max(1, std::min(kWave / L, kBandLds / tab->H))}
                           : BandOut{nullptr, 0, 0, 0, 1};
  if (fused && split)
    cws_kernel<true, true><<<sgrid, 256, 0, stream>>>(codes, counts, hist_off, n_distinct, N, t, hv, err, bo);
  else if (fused)
    cws_kernel<true, false><<<grid, 256, 0, stream>>>(codes, counts, hist_off, n_distinct, N, t, hv, err, bo);
  else if (split)
    cws_kernel<false, true><<<sgrid, 256, 0, stream>>>(codes, counts, hist_off, n_distinct, N, t, hv, err, bo);
  else
    cws_kernel<false, false><<<grid, 256, 0, stream>>>(codes, counts, hist_off, n_distinct, N, t, hv, err, bo);
  ssh_status st = check_launch("ssh_cws");
  if (st != SSH_OK || keys == nullptr || fused) return st;
  return band_keys_launch(hv, N, K, L, seed, keys, stream);
}

}  // namespace ssh
