// Weighted set of length-n bit shingles (Section 4.2, eq. "set").
//
// One wavefront per series.  The 2^n-token universe is a bitmap in LDS with a
// one-bit-per-word summary above it:
//   1. the series' stream words are staged in LDS; every shingle position
//      sets the bit of its token and the summary bit of that bitmap word
//      (LDS atomic ORs);
//   2. a wave prefix sum over the summary lists the occupied bitmap words in
//      order, and a prefix sum of their popcounts gives each word the rank of
//      its first token, so the distinct tokens come out in ascending order
//      without scanning the empty part of the universe;
//   3. every position adds one to the count of its token's rank (LDS
//      atomics; global atomics when a series has more distinct tokens than
//      the LDS count buffer holds);
//   4. only the words that were set are cleared for the next series.
// A token is the n bits in stream order read most significant first.
#include "common.hpp"

namespace ssh {

constexpr int kCountCap = 1024;
constexpr int kWordCap = 64;  // stream words staged in LDS per series

struct ShLds {
  uint32_t* bm;    // bitmap, BW words
  uint32_t* sm;    // summary, SW words
  uint32_t* pre;   // rank of the first token of each occupied word
  uint32_t* cnt;   // counts by rank
  uint16_t* list;  // occupied bitmap words, ascending
  uint64_t* wb;    // staged stream words
};

__device__ __forceinline__ uint32_t token_from(const uint64_t* wb, int p, int n) {
  const int wi = p >> 6, sh = p & 63;
  uint64_t v = wb[wi] >> sh;
  if (sh + n > 64) v |= wb[wi + 1] << (64 - sh);
  const uint32_t low = (uint32_t)v & (uint32_t)((1ull << n) - 1);
  return __builtin_bitreverse32(low) >> (32 - n);
}

__host__ __device__ inline size_t shingle_lds_words(int BW, int SW) {
  // staged words (u64), bitmap, summary, ranks, counts, list (u16), rounded to 8 bytes
  size_t w = (size_t)2 * kWordCap + BW + SW + BW + kCountCap + (BW + 1) / 2;
  return (w + 1) & ~(size_t)1;
}

__global__ __launch_bounds__(256) void shingle_kernel(const uint64_t* __restrict__ bits,
                                                      const int64_t* __restrict__ bit_word_off,
                                                      const int32_t* __restrict__ nbits, int64_t N,
                                                      int n, uint32_t* __restrict__ codes,
                                                      uint32_t* __restrict__ counts,
                                                      const int64_t* __restrict__ hist_off,
                                                      int32_t* __restrict__ n_distinct, int* err) {
  extern __shared__ uint64_t smem64[];
  const int BW = (1 << n) > 32 ? (1 << n) / 32 : 1;  // bitmap words
  const int SW = BW > 32 ? BW / 32 : 1;              // summary words
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  uint32_t* base = reinterpret_cast<uint32_t*>(smem64) + shingle_lds_words(BW, SW) * w;
  ShLds L;
  L.wb = reinterpret_cast<uint64_t*>(base);
  L.bm = base + 2 * kWordCap;
  L.sm = L.bm + BW;
  L.pre = L.sm + SW;
  L.cnt = L.pre + BW;
  L.list = reinterpret_cast<uint16_t*>(L.cnt + kCountCap);
  for (int i = lane; i < BW; i += kWave) L.bm[i] = 0;
  for (int i = lane; i < SW; i += kWave) L.sm[i] = 0;
  wave_sync_lds();

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
    const int nw = (nb + 63) / 64;
    if (hist_off[s + 1] - ho < S || bit_word_off[s + 1] - wo < nw) {
      if (lane == 0) {
        atomicOr(err, 1);
        n_distinct[s] = 0;
      }
      continue;
    }
    const uint64_t* wb = bits + wo;
    if (nw <= kWordCap) {
      if (lane < nw) L.wb[lane] = wb[lane];
      wave_sync_lds();
      wb = L.wb;
    }
    // 1. mark tokens and their bitmap words
    for (int p = lane; p < S; p += kWave) {
      const uint32_t t = token_from(wb, p, n);
      const uint32_t word = t >> 5;
      atomicOr(L.bm + word, 1u << (t & 31));
      atomicOr(L.sm + (word >> 5), 1u << (word & 31));
    }
    wave_sync_lds();
    // 2. occupied words in ascending order, then token ranks
    uint32_t nz = 0;
    for (int bi = 0; bi < SW; bi += kWave) {
      const int i = bi + lane;
      const uint32_t smw = i < SW ? L.sm[i] : 0u;
      const uint32_t c = __builtin_popcount(smw);
      const uint32_t incl = wave_incl_scan(c);
      uint32_t pos = nz + incl - c;
      uint32_t b = smw;
      while (b) {
        const int tb = __builtin_ctz(b);
        L.list[pos++] = (uint16_t)(i * 32 + tb);
        b &= b - 1;
      }
      nz += wave_bcast(incl, kWave - 1);
    }
    wave_sync_lds();
    uint32_t D = 0;
    for (uint32_t bi = 0; bi < nz; bi += kWave) {
      const uint32_t i = bi + lane;
      const uint32_t word = i < nz ? L.list[i] : 0u;
      const uint32_t b0 = i < nz ? L.bm[word] : 0u;
      const uint32_t c = __builtin_popcount(b0);
      const uint32_t incl = wave_incl_scan(c);
      uint32_t rk = D + incl - c;
      if (i < nz) L.pre[word] = rk;
      uint32_t b = b0;
      while (b) {
        const int tb = __builtin_ctz(b);
        codes[ho + rk] = word * 32u + (uint32_t)tb;
        ++rk;
        b &= b - 1;
      }
      D += wave_bcast(incl, kWave - 1);
    }
    // 3. counts by rank
    const bool in_lds = D <= (uint32_t)kCountCap;
    if (in_lds) {
      for (uint32_t i = lane; i < D; i += kWave) L.cnt[i] = 0;
    } else {
      for (uint32_t i = lane; i < D; i += kWave) counts[ho + i] = 0;
      // this wave's zero stores complete before its atomics below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
    wave_sync_lds();
    for (int p = lane; p < S; p += kWave) {
      const uint32_t t = token_from(wb, p, n);
      const uint32_t word = t >> 5, b = t & 31;
      const uint32_t rank = L.pre[word] + __builtin_popcount(L.bm[word] & ((1u << b) - 1u));
      if (in_lds) atomicAdd(L.cnt + rank, 1u);
      else atomicAdd(counts + ho + rank, 1u);
    }
    wave_sync_lds();
    if (in_lds)
      for (uint32_t i = lane; i < D; i += kWave) counts[ho + i] = L.cnt[i];
    // 4. clear what was set
    for (uint32_t i = lane; i < nz; i += kWave) L.bm[L.list[i]] = 0;
    for (int i = lane; i < SW; i += kWave) L.sm[i] = 0;
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
  const int SW = BW > 32 ? BW / 32 : 1;
  const int wpb = n >= 16 ? 2 : 4;  // keep a block's LDS within 64 KiB
  const size_t shm = (size_t)wpb * shingle_lds_words(BW, SW) * sizeof(uint32_t);
  shingle_kernel<<<grid_for(N, wpb, 1 << 16), wpb * kWave, shm, stream>>>(
      bits, bit_word_off, nbits, N, n, codes, counts, hist_off, n_distinct, err);
  return check_launch("ssh_shingle");
}

}  // namespace ssh
