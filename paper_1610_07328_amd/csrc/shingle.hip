// Weighted set of length-n bit shingles (Section 4.2, eq. "set").
//
// One wavefront per series.  The 2^n-token universe is a bitmap in LDS:
//   1. every shingle position sets the bit of its token (LDS atomic OR);
//   2. a wave prefix sum of per-word popcounts gives each occupied token its
//      rank, so the distinct tokens come out in ascending order;
//   3. every position adds one to the count of its token's rank (LDS
//      atomics; global atomics if a series has more distinct tokens than the
//      LDS count buffer holds);
//   4. the bits that were set are cleared again for the next series.
// A token is the n bits in stream order read most significant first.
#include "common.hpp"

namespace ssh {

constexpr int kCountCap = 1024;

__device__ __forceinline__ uint32_t token_at(const uint64_t* __restrict__ wb, int p, int n) {
  const int wi = p >> 6, sh = p & 63;
  uint64_t v = wb[wi] >> sh;
  if (sh + n > 64) v |= wb[wi + 1] << (64 - sh);
  const uint32_t low = (uint32_t)v & (uint32_t)((1ull << n) - 1);
  return __builtin_bitreverse32(low) >> (32 - n);
}

__global__ __launch_bounds__(256) void shingle_kernel(const uint64_t* __restrict__ bits,
                                                      const int64_t* __restrict__ bit_word_off,
                                                      const int32_t* __restrict__ nbits, int64_t N,
                                                      int n, uint32_t* __restrict__ codes,
                                                      uint32_t* __restrict__ counts,
                                                      const int64_t* __restrict__ hist_off,
                                                      int32_t* __restrict__ n_distinct, int* err) {
  extern __shared__ uint32_t smem[];
  const int BW = (1 << n) > 32 ? (1 << n) / 32 : 1;  // bitmap words
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* bm = smem + (size_t)w * (2 * BW + kCountCap);
  uint32_t* pre = bm + BW;
  uint32_t* cnt = pre + BW;
  for (int i = lane; i < BW; i += kWave) bm[i] = 0;
  wave_sync_lds();
  const int WPL = (BW + kWave - 1) / kWave;

  const int wpb = blockDim.x / kWave;
  for (int64_t s = (int64_t)blockIdx.x * wpb + w; s < N; s += (int64_t)gridDim.x * wpb) {
    const int nb = nbits[s];
    const int S = nb >= n ? nb - n + 1 : 0;
    const int64_t ho = hist_off[s];
    if (S == 0) {
      if (lane == 0) n_distinct[s] = 0;
      continue;
    }
    const int64_t wo = bit_word_off[s];
    if (hist_off[s + 1] - ho < S || bit_word_off[s + 1] - wo < (nb + 63) / 64) {
      if (lane == 0) {
        atomicOr(err, 1);
        n_distinct[s] = 0;
      }
      continue;
    }
    const uint64_t* wb = bits + wo;
    for (int p = lane; p < S; p += kWave) {
      const uint32_t t = token_at(wb, p, n);
      atomicOr(bm + (t >> 5), 1u << (t & 31));
    }
    wave_sync_lds();
    // ranks: exclusive prefix of popcounts in word order
    uint32_t mine = 0;
    for (int i = 0; i < WPL; ++i) {
      const int idx = lane * WPL + i;
      if (idx < BW) mine += __builtin_popcount(bm[idx]);
    }
    const uint32_t incl = wave_incl_scan(mine);
    const uint32_t D = wave_bcast(incl, kWave - 1);
    uint32_t run = incl - mine;
    for (int i = 0; i < WPL; ++i) {
      const int idx = lane * WPL + i;
      if (idx < BW) {
        uint32_t b = bm[idx];
        pre[idx] = run;
        uint32_t rk = run;
        run += __builtin_popcount(b);
        while (b) {
          const int t = __builtin_ctz(b);
          codes[ho + rk] = (uint32_t)idx * 32u + (uint32_t)t;
          ++rk;
          b &= b - 1;
        }
      }
    }
    const bool in_lds = D <= (uint32_t)kCountCap;
    if (in_lds) {
      for (uint32_t i = lane; i < D; i += kWave) cnt[i] = 0;
    } else {
      for (uint32_t i = lane; i < D; i += kWave) counts[ho + i] = 0;
      __threadfence();
    }
    wave_sync_lds();
    for (int p = lane; p < S; p += kWave) {
      const uint32_t t = token_at(wb, p, n);
      const uint32_t word = t >> 5, b = t & 31;
      const uint32_t rank = pre[word] + __builtin_popcount(bm[word] & ((1u << b) - 1u));
      if (in_lds) atomicAdd(cnt + rank, 1u);
      else atomicAdd(counts + ho + rank, 1u);
    }
    wave_sync_lds();
    if (in_lds)
      for (uint32_t i = lane; i < D; i += kWave) counts[ho + i] = cnt[i];
    for (int p = lane; p < S; p += kWave) bm[token_at(wb, p, n) >> 5] = 0;
    wave_sync_lds();
    if (lane == 0) n_distinct[s] = (int32_t)D;
  }
}

__device__ int g_shingle_err;

int take_shingle_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_shingle_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_shingle_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

ssh_status shingle_launch(const uint64_t* bits, const int64_t* bit_word_off, const int32_t* nbits,
                          int64_t N, int n, uint32_t* codes, uint32_t* counts,
                          const int64_t* hist_off, int32_t* n_distinct, hipStream_t stream) {
  if (N == 0) return SSH_OK;
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_shingle_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_shingle: cannot resolve error flag");
  const int BW = (1 << n) > 32 ? (1 << n) / 32 : 1;
  const int wpb = n >= 16 ? 2 : 4;  // keep a block's LDS within 64 KiB
  const size_t shm = (size_t)wpb * (2 * BW + kCountCap) * sizeof(uint32_t);
  shingle_kernel<<<grid_for(N, wpb, 1 << 16), wpb * kWave, shm, stream>>>(
      bits, bit_word_off, nbits, N, n, codes, counts, hist_off, n_distinct, err);
  return check_launch("ssh_shingle");
}

}  // namespace ssh
