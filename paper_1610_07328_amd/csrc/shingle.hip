// Weighted set of length-n bit shingles (Section 4.2, eq. "set").
//
// One wavefront per series; lane L takes P consecutive shingle positions
// (P = ceil(S / 64), at most 33 - n, in rounds when the series is longer).
// The P + n - 1 stream bits a lane needs sit in one 32-bit window; after a
// bit reversal, the token at position b0 + k is the n-bit field at offset
// 32 - n - k, so every token costs one bit-field extract.
//   1. every lane sets its tokens' bits in a 2^n-bit LDS bitmap (LDS atomic
//      OR, skipped when a token repeats the lane's previous one);
//   2. each lane owns 2^n / 2048 consecutive bitmap words: their popcounts,
//      a wave prefix sum and a running sum give every word the rank of its
//      first token (16-bit), and the total is the number D of distinct tokens;
//   3. each token's rank is its word's base plus the popcount of the lower
//      bits of its word; runs of equal tokens inside a lane are counted once
//      with their length (LDS atomic add on 16-bit halves, or a global one
//      when D exceeds the LDS count buffer or the series has 2^16 shingles or
//      more), and the token is written at its rank of `codes`,
//      so tokens come out ascending without sorting;
//   4. counts are copied out and the bitmap and counts are cleared.
// Lane L's bitmap words sit in a padded per-lane run, read and cleared with
// 16-byte LDS accesses that fall on distinct banks; for n >= 13 the padding
// holds the lane's rank bases, so the wave's LDS stays small (6 KB at n = 15)
// and more waves fit a CU.
// A token is the n bits in stream order read most significant first.
#include <climits>
#include <type_traits>

#include "common.hpp"

namespace ssh {

// Distinct tokens whose counts stay in LDS, two 16-bit counts per 32-bit word
// (exact while the series has fewer than 2^16 shingles, the only case that
// uses them: every count is at most the shingle count).  Series of at most
// kCountCap shingles (so at most that many distinct tokens) run in one launch
// with this buffer; longer ones in a second launch whose buffer holds
// kCountCapLong, so that a long series' counts stay in LDS too without the
// short series' launch giving up occupancy for it.
constexpr int kCountCap = 512;
constexpr int kCountCapLong = 2048;
constexpr int kShWaves = 1;     // wavefronts per workgroup

__host__ __device__ inline int shingle_bitmap_words(int n) { return n > 5 ? 1 << (n - 5) : 1; }
__host__ __device__ inline int shingle_wpl(int n) {  // bitmap words per lane
  const int bw = shingle_bitmap_words(n);
  return bw >= kWave ? bw / kWave : 1;
}
// Lane L owns bitmap words [L WPL, (L + 1) WPL), stored from slot L BS; the
// stride is padded so that the lanes' 16-byte accesses of one instruction
// fall on distinct LDS banks.  With WPL >= 8 the four padding words hold the
// lane's rank bases: 8 u16, one per group of WPL / 8 words.  With fewer words
// per lane the bases (one per word) sit in an array of their own.
__host__ __device__ constexpr int shingle_bs(int wpl) { return wpl + (wpl >= 8 ? 4 : 0); }
__host__ __device__ constexpr int shingle_pre_u16(int wpl) { return wpl >= 8 ? 0 : kWave * wpl; }

// LDS bytes of one wave (set by the words per lane: every n <= 11 has one):
// bitmap (u32) and rank bases, separate bases (u16, to 16 bytes), counts
// (u16).  The kernel's LDS is a static array of this size, so its addresses
// are constants the instructions fold in.
__host__ __device__ constexpr int shingle_lds_bytes(int wpl, int cap) {
  return kWave * shingle_bs(wpl) * 4 + ((shingle_pre_u16(wpl) * 2 + 15) & ~15) + cap * 2;
}

// 32 stream bits starting at bit b0 (bit j of the result is stream bit b0 + j),
// through a buffer resource over the series' stream words: words past its
// range read as zero
__device__ __forceinline__ uint32_t stream_window(__amdgpu_buffer_rsrc_t ws, int b0) {
  const int i = b0 >> 5;
  const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b32(ws, 4 * i, 0, 0);
  const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b32(ws, 4 * i + 4, 0, 0);
  return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(b0 & 31));
}

// Inclusive prefix sum over the wave by DPP: Hillis-Steele shifts inside each
// row of 16 lanes, then the row totals through row_bcast:15 and row_bcast:31.
// Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
  return v;
}

// CAP: the LDS count capacity; the launch hashes the series whose shingle
// count S lies in [s_lo, s_hi] (and records n_distinct only for those)
template <int WPL, int CAP>
__global__ __launch_bounds__(kShWaves * kWave) void shingle_kernel(
    const uint64_t* __restrict__ bits, const int64_t* __restrict__ bit_word_off,
    const int32_t* __restrict__ nbits, int64_t N, int n, uint32_t* __restrict__ codes,
    uint32_t* __restrict__ counts, const int64_t* __restrict__ hist_off,
    int32_t* __restrict__ n_distinct, int* err, int s_lo, int s_hi) {
  constexpr int BS = WPL + (WPL >= 8 ? 4 : 0);    // shingle_bs
  constexpr bool PAD = WPL >= 8;                  // rank bases in the padding words
  constexpr int GS = PAD ? WPL / 8 : 1;           // words per rank base
  constexpr int LW = WPL == 1 ? 0 : (WPL == 2 ? 1 : (WPL == 4 ? 2 : (WPL == 8 ? 3 : (WPL == 16 ? 4 : 5))));
  __shared__ __attribute__((aligned(16))) uint32_t smem32[kShWaves * shingle_lds_bytes(WPL, CAP) / 4];
  const int BW = shingle_bitmap_words(n);
  // wave-uniform; a constant 0 for one-wave workgroups, so LDS addresses
  // fold their base into instruction offsets
  const int w = kShWaves == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  uint32_t* bm = smem32 + (shingle_lds_bytes(WPL, CAP) / 4) * w;
  uint16_t* pre = reinterpret_cast<uint16_t*>(bm + kWave * BS);  // separate bases (!PAD)
  uint32_t* cnt = bm + kWave * BS + ((shingle_pre_u16(WPL) * 2 + 15) & ~15) / 4;
  // this lane's words exist (WPL > 1: the bitmap is exactly 64 WPL words)
  const bool own = WPL > 1 || lane < BW;
  uint32_t* mybm = bm + lane * BS;
  uint16_t* mypre = PAD ? reinterpret_cast<uint16_t*>(mybm + WPL) : pre + lane * WPL;
  for (int i = lane; i < kWave * BS; i += kWave) bm[i] = 0;
  for (int i = lane; i < CAP / 2; i += kWave) cnt[i] = 0;
  wave_sync_lds();
  const uint32_t mask = (1u << n) - 1u;  // n <= 16
  // slot of word wd, and the rank of its first token
  auto bslot = [&](uint32_t wd) { return (int)((wd >> LW) * BS + (wd & (WPL - 1))); };
  auto word_rank = [&](uint32_t wd) -> uint32_t {
    const int j = (int)(wd & (WPL - 1));
    if constexpr (PAD) {
      const uint32_t* run = bm + (wd >> LW) * BS;
      uint32_t r = reinterpret_cast<const uint16_t*>(run + WPL)[j / GS];
      if constexpr (GS > 1) {
        // the words of the group before word j, read unconditionally (they
        // are in the lane's run) and counted when they precede j
        const int j0 = j - j % GS;
#pragma unroll
        for (int i = 0; i < GS - 1; ++i) {
          const uint32_t c = __builtin_popcount(run[j0 + i]);
          r += j0 + i < j ? c : 0u;
        }
      }
      return r;
    } else {
      return pre[(wd >> LW) * WPL + j];
    }
  };

  // The wave's series are s0 + k stride, k = 0, 1, ...  It reads the bit
  // counts of 64 of them at once (one per lane) and takes, in order, those
  // whose shingle count this launch handles, so skipping the other launch's
  // series costs no chain of dependent loads.
  const int64_t s0 = (int64_t)blockIdx.x * kShWaves + w;
  const int64_t stride = (int64_t)gridDim.x * kShWaves;
  for (int64_t k0 = 0; s0 + k0 * stride < N; k0 += kWave) {
    const int64_t sl = s0 + (k0 + lane) * stride;
    const int nbl = sl < N ? nbits[sl] : 0;
    const int Sl = nbl >= n ? nbl - n + 1 : 0;
    uint64_t todo = ballot64(sl < N && Sl >= s_lo && Sl <= s_hi);
    while (todo) {
      const int j = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int64_t s = s0 + (k0 + j) * stride;
      const int nb = __builtin_amdgcn_readlane(nbl, j);
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
      const __amdgpu_buffer_rsrc_t ws = __builtin_amdgcn_make_buffer_rsrc(
          (void*)(bits + wo), 0, 8 * nw, 0x00020000);
      uint32_t* const codes_s = codes + ho;
      uint32_t* const counts_s = counts + ho;
      int P = (S + kWave - 1) / kWave;
      if (P > 33 - n) P = 33 - n;
      const int per_round = kWave * P;

      // 1. mark the tokens (the first round's stream window is kept for step 3)
      uint32_t rev0 = 0;
      for (int base = 0; base < S; base += per_round) {
        const int b0 = base + lane * P;
        if (b0 < S) {
          const uint32_t rev = __builtin_bitreverse32(stream_window(ws, b0));
          if (base == 0) rev0 = rev;
          const int kend = S - b0 < P ? S - b0 : P;
          uint32_t prev = 0xFFFFFFFFu;
          for (int k = 0; k < kend; ++k) {
            const uint32_t t = (rev >> (32 - n - k)) & mask;
            if (t != prev) atomicOr(bm + bslot(t >> 5), 1u << (t & 31));
            prev = t;
          }
        }
      }
      wave_sync_lds();

      // 2. rank of the first token of every bitmap word, and D
      uint32_t wv[WPL];
      if constexpr (WPL >= 4) {
  #pragma unroll
        for (int q = 0; q < WPL / 4; ++q) {
          const uint4 v = reinterpret_cast<const uint4*>(mybm)[q];
          wv[4 * q] = v.x; wv[4 * q + 1] = v.y; wv[4 * q + 2] = v.z; wv[4 * q + 3] = v.w;
        }
      } else if constexpr (WPL == 2) {
        const uint2 v = reinterpret_cast<const uint2*>(mybm)[0];
        wv[0] = v.x; wv[1] = v.y;
      } else {
        wv[0] = own ? mybm[0] : 0u;
      }
      uint32_t c = 0;
  #pragma unroll
      for (int j = 0; j < WPL; ++j) c += __builtin_popcount(wv[j]);
      const uint32_t incl = wave_incl_scan_dpp(c);
      uint32_t rk = incl - c;
      uint16_t pv[WPL];
  #pragma unroll
      for (int j = 0; j < WPL; ++j) {
        pv[j] = (uint16_t)rk;
        rk += __builtin_popcount(wv[j]);
      }
      if constexpr (PAD) {
        // the bases of word groups 0, GS, 2 GS, ... into the padding words
        uint4 v;
        v.x = pv[0] | ((uint32_t)pv[GS] << 16);
        v.y = pv[2 * GS] | ((uint32_t)pv[3 * GS] << 16);
        v.z = pv[4 * GS] | ((uint32_t)pv[5 * GS] << 16);
        v.w = pv[6 * GS] | ((uint32_t)pv[7 * GS] << 16);
        reinterpret_cast<uint4*>(mypre)[0] = v;
      } else if constexpr (WPL == 4) {
        reinterpret_cast<uint2*>(mypre)[0] =
            make_uint2(pv[0] | ((uint32_t)pv[1] << 16), pv[2] | ((uint32_t)pv[3] << 16));
      } else if constexpr (WPL == 2) {
        reinterpret_cast<uint32_t*>(mypre)[0] = pv[0] | ((uint32_t)pv[1] << 16);
      } else {
        if (own) mypre[0] = pv[0];
      }
      const uint32_t D = __builtin_amdgcn_readlane(incl, kWave - 1);
      const bool in_lds = D <= (uint32_t)CAP && S < 65536;
      if (!in_lds) {
        for (uint32_t i = lane; i < D; i += kWave) counts_s[i] = 0;
        // this wave's zero stores complete before its atomics below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      }
      wave_sync_lds();

      // 3. counts by rank (runs of equal tokens in a lane counted at once), codes
      // at their ranks; counts in LDS or (more than CAP tokens) in memory,
      // two copies of the loop so that each uses its own kind of atomic
      auto step3 = [&](auto lds_counts) {
        constexpr bool LDS_COUNTS = decltype(lds_counts)::value;
        auto flush = [&](uint32_t t, uint32_t run) {
          const uint32_t wd = t >> 5;
          uint32_t rank;
          if constexpr (GS == 2) {
            // the token's word and its group partner are one aligned 64-bit
            // pair; t's bit sits at position t mod 64 of the pair and is set,
            // so shifting it to the top leaves it and the lower bits
            const uint32_t* run_w = bm + (wd >> LW) * BS;
            const uint32_t g = (wd & (WPL - 1)) >> 1;
            const uint2 pr = reinterpret_cast<const uint2*>(run_w)[g];
            const uint32_t base = reinterpret_cast<const uint16_t*>(run_w + WPL)[g];
            const uint64_t v = ((uint64_t)pr.y << 32 | pr.x) << ((t ^ 63u) & 63u);
            rank = base + (uint32_t)__builtin_popcountll(v) - 1u;
          } else {
            rank = word_rank(wd) + __builtin_popcount(bm[bslot(wd)] & ((1u << (t & 31)) - 1u));
          }
          if constexpr (LDS_COUNTS) atomicAdd(cnt + (rank >> 1), run << ((rank & 1u) * 16u));
          else atomicAdd(counts_s + rank, run);
          codes_s[rank] = t;
        };
        for (int base = 0; base < S; base += per_round) {
          const int b0 = base + lane * P;
          if (b0 < S) {
            const uint32_t rev =
                base == 0 ? rev0 : __builtin_bitreverse32(stream_window(ws, b0));
            const int kend = S - b0 < P ? S - b0 : P;
            uint32_t prev = (rev >> (32 - n)) & mask;
            uint32_t run = 1;
            for (int k = 1; k < kend; ++k) {
              const uint32_t t = (rev >> (32 - n - k)) & mask;
              if (t == prev) {
                ++run;
                continue;
              }
              flush(prev, run);
              prev = t;
              run = 1;
            }
            flush(prev, run);
          }
        }
      };
      if (in_lds) step3(std::true_type{});
      else step3(std::false_type{});
      wave_sync_lds();

      // 4. counts out; clear the bitmap words and counts that were used
      if (in_lds) {
        for (uint32_t i = lane; i < D; i += kWave) counts_s[i] = (cnt[i >> 1] >> ((i & 1u) * 16u)) & 0xFFFFu;
        wave_sync_lds();
        for (uint32_t i = lane; i < (D + 1) / 2; i += kWave) cnt[i] = 0;
      }
      if constexpr (WPL >= 4) {
  #pragma unroll
        for (int q = 0; q < WPL / 4; ++q) reinterpret_cast<uint4*>(mybm)[q] = make_uint4(0u, 0u, 0u, 0u);
      } else if constexpr (WPL == 2) {
        reinterpret_cast<uint2*>(mybm)[0] = make_uint2(0u, 0u);
      } else {
        if (own) mybm[0] = 0u;
      }
      wave_sync_lds();
      if (lane == 0) n_distinct[s] = (int32_t)D;
    }
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
  const int wpl = shingle_wpl(n);
  const unsigned grid = grid_for(N, kShWaves, 1 << 16);
  const dim3 block(kShWaves * kWave);
  // series of up to kCountCap shingles, then the longer ones
#define SSH_SHINGLE_CASE(V)                                                                     \
  case V:                                                                                       \
    shingle_kernel<V, kCountCap><<<grid, block, 0, stream>>>(                                   \
        bits, bit_word_off, nbits, N, n, codes, counts, hist_off, n_distinct, err, 0,           \
        kCountCap);                                                                             \
    shingle_kernel<V, kCountCapLong><<<grid, block, 0, stream>>>(                               \
        bits, bit_word_off, nbits, N, n, codes, counts, hist_off, n_distinct, err,              \
        kCountCap + 1, INT_MAX);                                                                \
    break;
  switch (wpl) {
    SSH_SHINGLE_CASE(1)
    SSH_SHINGLE_CASE(2)
    SSH_SHINGLE_CASE(4)
    SSH_SHINGLE_CASE(8)
    SSH_SHINGLE_CASE(16)
    SSH_SHINGLE_CASE(32)
    default:
      return fail(SSH_EUNSUPPORTED, "ssh_shingle: n outside [1, 16]");
  }
#undef SSH_SHINGLE_CASE
  return check_launch("ssh_shingle");
}

}  // namespace ssh
