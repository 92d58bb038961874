// Weighted MinHash by integer replication (Section 2, eqs. WJaccardDef and
// CollProb; the one-pass minimum of Section 4, Discussions and Practical Issues).
//
// With integer weights, a weighted set {(c, n_c)} is the plain set of pairs
// (c, j), j = 1..n_c, and a min-hash over those pairs collides between two
// series with probability sum_c min(n_c, m_c) / sum_c max(n_c, m_c), the
// generalized Jaccard similarity.  Hash k ranks a pair by
//     v_k(c, j) = mix(s_k ^ (c << 32 | j)),  s_k = mix(seed + (k + 1) gamma),
// mix the SplitMix64 output function, gamma = 0x9E3779B97F4A7C15, and the
// hash value is the pair (c << 32 | j) of smallest v_k; equal v_k resolve to
// the pair met first in input order (token order, then j ascending).  No
// floating point is involved, so the result is exact by construction.
//
// One wavefront per series.  Lane L holds the running minima of hashes L and
// L + 64 of a group of 128 (a last group of at most 64 hashes takes one per
// lane); H > 128 loops over groups and re-reads the tokens from cache.  Tokens are loaded 64 at a time, one per
// lane, and broadcast with readlane, so the pair loop is wave-uniform and
// every active lane does one 64-bit mix per pair and hash.
#include "band.hpp"
#include "common.hpp"

namespace ssh {

constexpr int kWmhWaves = 4;
constexpr uint64_t kMixC1 = 0xBF58476D1CE4E5B9ull;  // SplitMix64 output multipliers
constexpr uint64_t kMixC2 = 0x94D049BB133111EBull;

// mix(s ^ (c << 32 | j)) for one token c, the high word of the argument
// (s_hi ^ c) fixed: the first round's shift of the high word and its share
// of the first product's high word are taken once per token.
struct TokMix {
  uint32_t zhi;  // s_hi ^ c
  uint32_t kc;   // low word of (zhi ^ zhi >> 30) * C1_lo
  uint32_t slo;  // s_lo
};

__device__ __forceinline__ TokMix tok_mix(uint64_t s, uint32_t c) {
  TokMix t;
  t.zhi = (uint32_t)(s >> 32) ^ c;
  t.kc = (t.zhi ^ (t.zhi >> 30)) * (uint32_t)kMixC1;
  t.slo = (uint32_t)s;
  return t;
}

__device__ __forceinline__ uint64_t elem_mix(const TokMix& t, uint32_t j) {
  const uint32_t zlo = t.slo ^ j;
  const uint32_t tlo = zlo ^ ((zlo >> 30) | (t.zhi << 2));  // low word of z ^ z >> 30
  const uint64_t p = (uint64_t)tlo * (uint32_t)kMixC1;
  const uint32_t phi = (uint32_t)(p >> 32) + tlo * (uint32_t)(kMixC1 >> 32) + t.kc;
  uint64_t z = (uint64_t)phi << 32 | (uint32_t)p;
  z = (z ^ (z >> 27)) * kMixC2;
  return z ^ (z >> 31);
}

// Hashes k0 + lane and, with TWO, k0 + 64 + lane of one series: the running
// minimum over its elements in input order, stored to row[k] for k < H.
template <bool TWO>
__device__ __forceinline__ void wmh_group(const uint32_t* __restrict__ codes,
                                          const uint32_t* __restrict__ counts, int64_t off, int d,
                                          uint64_t seed, int k0, int H, uint64_t* __restrict__ row) {
  const int lane = lane_id();
  const int ka = k0 + lane, kb = k0 + kWave + lane;
  const uint64_t sa = mix64(seed + (uint64_t)(ka + 1) * 0x9E3779B97F4A7C15ull);
  const uint64_t sb = TWO ? mix64(seed + (uint64_t)(kb + 1) * 0x9E3779B97F4A7C15ull) : 0;
  uint64_t va = ~0ull, vb = ~0ull, ia = SSH_HV_EMPTY, ib = SSH_HV_EMPTY;
  bool have = false;  // wave-uniform: some element has been seen
  for (int t0 = 0; t0 < d; t0 += kWave) {
    const int nt = d - t0 < kWave ? d - t0 : kWave;
    const uint32_t myc = lane < nt ? codes[off + t0 + lane] : 0u;
    const uint32_t myn = lane < nt ? counts[off + t0 + lane] : 0u;
    for (int t = 0; t < nt; ++t) {
      const uint32_t c = __builtin_amdgcn_readlane(myc, t);
      const uint32_t n = __builtin_amdgcn_readlane(myn, t);
      if (!have && n > 0) {
        // the first element seeds the minima, so an element whose rank is
        // all ones still wins when nothing smaller follows (the loop below
        // meets it again with an equal rank, which changes nothing)
        const uint64_t key = (uint64_t)c << 32 | 1u;
        va = mix64(sa ^ key);
        ia = key;
        if (TWO) {
          vb = mix64(sb ^ key);
          ib = key;
        }
        have = true;
      }
      const TokMix ta = tok_mix(sa, c), tb = tok_mix(sb, c);
      // j = 1 .. n, wave-uniform; the test also ends the loop for n = 2^32 - 1
      for (uint32_t j = 1; j - 1u < n; ++j) {
        const uint64_t wa = elem_mix(ta, j);
        if (wa < va) { va = wa; ia = (uint64_t)c << 32 | j; }
        if (TWO) {
          const uint64_t wb = elem_mix(tb, j);
          if (wb < vb) { vb = wb; ib = (uint64_t)c << 32 | j; }
        }
      }
    }
  }
  if (ka < H) row[ka] = ia;
  if (TWO && kb < H) row[kb] = ib;
}

// One wave per series; hashes in groups of 128 (two per lane), the last group
// of at most 64 with one per lane.
__global__ __launch_bounds__(kWave * kWmhWaves) void wmh_int_kernel(
    const uint32_t* __restrict__ codes, const uint32_t* __restrict__ counts,
    const int64_t* __restrict__ hist_off, const int32_t* __restrict__ n_distinct, int64_t N,
    int H, uint64_t seed, uint64_t* __restrict__ hv) {
  const int64_t wave0 = (int64_t)blockIdx.x * kWmhWaves + threadIdx.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWmhWaves;
  for (int64_t s = wave0; s < N; s += nwaves) {
    const int64_t off = hist_off[s];
    const int d = n_distinct[s];
    for (int k0 = 0; k0 < H; k0 += 2 * kWave) {
      if (H - k0 > kWave)
        wmh_group<true>(codes, counts, off, d, seed, k0, H, hv + s * H);
      else
        wmh_group<false>(codes, counts, off, d, seed, k0, H, hv + s * H);
    }
  }
}

ssh_status wmh_int_launch(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                          const int32_t* n_distinct, int64_t N, int H, uint64_t seed, uint64_t* hv,
                          hipStream_t stream) {
  if (N == 0) return SSH_OK;
  const int64_t want = (N + kWmhWaves - 1) / kWmhWaves;
  const int blocks = (int)(want < (1 << 20) ? want : (1 << 20));
  wmh_int_kernel<<<blocks, kWave * kWmhWaves, 0, stream>>>(codes, counts, hist_off, n_distinct, N, H,
                                                           seed, hv);
  return check_launch("ssh_wmh_int");
}

}  // namespace ssh
