// Sign sketches of several random filters at once: Section 4.1's sketch with
// F filters r_1 .. r_F in place of one, as a matrix product on the matrix
// cores.
//
// Bit (f, i) of a series = [ r_f . x[i delta .. i delta + W) >= 0 ]: F sign
// streams, stream f being exactly the single-filter sketch of filter r_f.  For
// a work item of 128 or 256 consecutive windows of one series the inner
// products are
//     S[f][w] = sum_k R[f][k] X[k][w],  R[f][k] = r_f[k],  X[k][w] = x[w delta + k]
// (filters x taps times taps x windows; taps padded to a multiple of the MFMA
// depth with zero filter entries).  The filters are the A operand, held in
// registers for the whole launch; the windows are the B operand, read from
// LDS, where the item's samples sit as fp16 quads starting at every sample
// (every second or fourth sample when delta is even or a multiple of 4), so
// that every window's run of consecutive samples is a run of whole quads
// whatever delta is.  One 16x16xK fp16 MFMA per 16 filters, 16 windows and K
// taps (fp16 products exact in fp32, fp32 accumulation).  Lane (g, n) of a
// product holds window n against filters 4 g .. 4 g + 3, so one ballot per
// element packs the signs of 16 windows for four filters at once.
//
// Exactness.  The reference bit is the sign of the float64 sum of exact
// products in ascending filter index.  With x^ = fp16(x) and margin weights
// c_k = |r^_k| (r^ = fp16(r)), the single-filter matrix path's derivation
// bounds the fast sum's distance from the reference sum by
// c1a sum_k c_k |x^_k| + c0a.  Here the L1 term is bounded once more, by
// Cauchy-Schwarz: sum_k c_k |x^_k| <= ||c|| ||x^_w||, with ||x^_w||^2 taken
// from the same fp16 fragments the MFMA reads (v_dot2 in fp32, every rounding
// covered by a factor 1 + 2^-12) plus 2^-14 sum c_k for samples in fp16's
// subnormal range, whatever the hardware does with them.  So a pair whose
// |S| > K1 ||x^_w|| + K0 (per-filter constants) keeps the sign of S, with no
// second matrix product.  A filter entry in fp16's subnormal range
// (0 < |r| < 2^-14) enters the product as 0 and its weight is raised to
// c_k >= 2^-14 (1 + v) / (2v + v^2) (v = 2^-11 / (1 - 2^-11)): its whole
// term |r_k x_k| <= 2^-14 |x_k| is then within the bound the margin grants
// every other entry, so every finite filter with |r| < 2^14 is covered.
// Untrusted pairs are queued in LDS and, before the item's words are
// stored, recomputed as the float64 sum of exact products from float32
// copies of the item's samples and of the filters held in LDS; an item
// holding a sample with |x| >= 2^14 or a non-finite one, or more untrusted
// pairs than the queue takes, is computed that way in full.
#include <cmath>
#include <cstring>
#include <vector>

#include "sketch_core.hpp"

namespace ssh {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));

struct MultiArgs {
  const float* r32;   // [F][WP] float32 filters, zero past W
  const uint2* rh;    // [F][WP / 4] fp16 quads of the filters (subnormal-range entries as 0)
  const float2* kst;  // [F] (K1, K0) of each filter's margin K1 ||x^_w|| + K0
  int WP;             // padded filter length (row stride of r32, 4 x that of rh)
  int fbase;          // first filter of this launch
};

constexpr int kQcapMulti = 512;          // queued (window, filter) pairs per item

// Sign of the float64 sum of exact products r[k] x[k], k ascending.
template <int W>
__device__ __forceinline__ bool exact_sign(const float* xw, const float* rf) {
  double acc = 0.0;
#pragma unroll 8
  for (int k = 0; k < W; ++k) acc = __builtin_fma((double)rf[k], (double)xw[k], acc);
  return acc >= 0.0;
}

// 16 filters x 16 windows x KW taps.  KW = 16: lane (g, n) supplies taps
// 4 g .. 4 g + 3 of its row / column; KW = 32: taps 8 g .. 8 g + 7.
template <int KW>
__device__ __forceinline__ float4v mfma_taps(const uint2 (&a)[KW / 16], const uint2 (&b)[KW / 16],
                                             float4v c) {
  if constexpr (KW == 16) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(half4, a[0]),
                                                 __builtin_bit_cast(half4, b[0]), c, 0, 0, 0);
  } else {
    const uint4 a4 = make_uint4(a[0].x, a[0].y, a[1].x, a[1].y);
    const uint4 b4 = make_uint4(b[0].x, b[0].y, b[1].x, b[1].y);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8, a4),
                                                  __builtin_bit_cast(half8, b4), c, 0, 0, 0);
  }
}

// x0^2 + x1^2 + acc for a pair of fp16 values
__device__ __forceinline__ float sq2(uint32_t u, float acc) {
  const h2 v = __builtin_bit_cast(h2, u);
  return __builtin_amdgcn_fdot2(v, v, acc, false);
}

// MT: 16-window tiles per work item (8 or 16); WPE: the waves per SIMD the
// register budget is fitted to (the item size and the budget set how many
// waves share a SIMD, through LDS and registers)
template <int W, int D, int KW, int NT, int MT, int WPE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void sketch_multi_kernel(
    const float* __restrict__ x, const int64_t* __restrict__ x_off, int64_t N, MultiArgs ma,
    uint64_t* __restrict__ bits, int64_t total_words, const int64_t* __restrict__ bit_word_off,
    int32_t* __restrict__ nbits_out, unsigned long long* repair_count, int* err) {
  constexpr int kMtItem = MT;                                // 16-window tiles per item
  constexpr int kSubMulti = 16 * MT;                         // windows per item
  constexpr int WP = (W + KW - 1) / KW * KW;                // padded taps
  constexpr int KS = WP / KW;                                // k-steps
  constexpr int QL = KW / 16;                                // quads per lane per k-step
  constexpr int FG = 16 * NT;                                // filters of this launch
  constexpr int NS = (kSubMulti - 1) * D + WP;               // samples an item reads
  constexpr int NC = D % 4 == 0 ? 1 : (D % 2 == 0 ? 2 : 4);  // quads per 4 samples
  constexpr int CSTEP = 4 / NC;                              // samples between quads
  constexpr int NQ = (NS + 3) / 4;                           // 4-sample groups staged
  constexpr int PF4 = (NS + 4 + 4 * kWave - 1) / (4 * kWave);  // 256-sample rows loaded
  constexpr int WPI = kMtItem / 2;                           // 32-bit words per filter per item
  static_assert(FG <= 256 && kSubMulti <= 256 && kSubMulti % 64 == 0,
                "queue entries are bytes; items hold whole stream words");

  constexpr int RS = W | 1;  // odd row stride: the rows of one tap sit on distinct banks
  __shared__ float rs[FG][RS];  // the launch's filters, float32
  // quad i = samples CSTEP i .. CSTEP i + 3 (fp16): every window's fragment
  // starts at a quad, and the 16 lanes of one fragment read fall on distinct
  // LDS banks for the shapes here
  __shared__ uint2 xq[kWavesPerBlock][NC * NQ];
  __shared__ __attribute__((aligned(16))) float xs[kWavesPerBlock][4 * NQ];  // float32 samples
  __shared__ uint8_t qwin[kWavesPerBlock][kQcapMulti];  // queued pair: item-relative window
  __shared__ uint8_t qfil[kWavesPerBlock][kQcapMulti];  //   and launch-relative filter
  // sign masks of the item: bm[nt][i][mt] bit 16 g + n = window 16 mt + n
  // against filter 16 nt + 4 g + i
  __shared__ uint64_t bm[kWavesPerBlock][NT][4][kMtItem];

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  const int n16 = lane & 15, g = lane >> 4;
  uint32_t* bits32 = reinterpret_cast<uint32_t*>(bits);
  // pairs this wave recomputed in float64, added to the global count once at
  // the end (one atomic per item on a single address would serialise)
  unsigned long long repaired = 0;

  for (int i = threadIdx.x; i < FG * W; i += blockDim.x) {
    const int fl = i / W, k = i - fl * W;
    rs[fl][k] = ma.r32[(int64_t)(ma.fbase + fl) * ma.WP + k];
  }
  __syncthreads();

  // A operands: lane (g, n) holds taps KW t + (KW / 4) g .. of filter
  // fbase + 16 nt + n; the product's element i of lane (g, n) belongs to
  // filter fbase + 16 nt + 4 g + i, whose margin constants the lane keeps
  uint2 rb[NT][KS][QL];
  float2 kk[NT][4];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int f = ma.fbase + 16 * nt + n16;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
#pragma unroll
      for (int j = 0; j < QL; ++j)
        rb[nt][t][j] = ma.rh[(int64_t)f * (ma.WP / 4) + (KW / 4) * t + QL * g + j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) kk[nt][i] = ma.kst[ma.fbase + 16 * nt + 4 * g + i];
  }

  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
  const int64_t s0 = (int64_t)blockIdx.x * kWavesPerBlock + w;
  ChunkItem cur;
  cur.s = N;
  if (s0 < N) {
    cur = series_item<W, D>(s0, x_off, bit_word_off, nbits_out, err);
    if (cur.nb == 0)
      cur = next_item<W, D, kSubMulti>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
  }
  float pv[PF4][4];
  if (cur.s < N) load_item4<PF4>(x, cur, (int64_t)cur.c * kSubMulti * D, pv);

  while (cur.s < N) {
    // stage the item's samples: float32 copies and fp16 quads, NC per 4
    // samples; flag the item when a sample could overflow the fp16 products
    // or is not finite
    bool bad = false;
#pragma unroll
    for (int i = 0; i < PF4; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) bad |= !(__builtin_fabsf(pv[i][e]) < 16384.0f);
    }
    const bool unsafe = ballot64(bad) != 0;
#pragma unroll
    for (int i = 0; i < PF4; ++i) {
      const int p = lane + kWave * i;  // this lane's 4-sample group
      if (p < NQ)
        *reinterpret_cast<float4*>(&xs[w][4 * p]) =
            make_float4(pv[i][0], pv[i][1], pv[i][2], pv[i][3]);
      if constexpr (NC == 1) {
        if (p < NQ)
          xq[w][p] = make_uint2(pack_f16(pv[i][0], pv[i][1]), pack_f16(pv[i][2], pv[i][3]));
      } else {
        // the group after this lane's: lane + 1's, or the next row's lane 0
        float v[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = pv[i][e];
          const float up = __shfl(pv[i][e], (lane + 1) & (kWave - 1), kWave);
          const float nx = i + 1 < PF4 ? __shfl(pv[i + 1 < PF4 ? i + 1 : i][e], 0, kWave) : 0.0f;
          v[4 + e] = lane == kWave - 1 ? nx : up;
        }
        if (p < NQ) {
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) {
            const int sh = cc * CSTEP;
            xq[w][NC * p + cc] = make_uint2(pack_f16(v[sh], v[sh + 1]), pack_f16(v[sh + 2], v[sh + 3]));
          }
        }
      }
    }
    wave_sync_lds();

    // start loading the next item; it is staged at the top of the next iteration
    const ChunkItem nxt =
        next_item<W, D, kSubMulti>(cur, N, stride, x_off, bit_word_off, nbits_out, err);
    if (nxt.s < N) load_item4<PF4>(x, nxt, (int64_t)nxt.c * kSubMulti * D, pv);

    const int nb_item = cur.nb - cur.c * kSubMulti;  // windows of the series from here on
    const int nwin = nb_item < kSubMulti ? nb_item : kSubMulti;
    int qc = 0;  // queued pairs of this item (wave-uniform)
    bool full = unsafe;
    if (!full) {
      // the B fragments of tile mt (this lane's window 16 mt + n)
      auto frags = [&](int mt, uint2 (&A)[KS][QL]) {
        const int wl = 16 * mt + n16;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
          const int st = wl * D + KW * t + (KW / 4) * g;  // first sample of the fragment
          const uint2* src = &xq[w][st / CSTEP];
#pragma unroll
          for (int j = 0; j < QL; ++j) A[t][j] = src[NC * j];  // samples st + 4 j ..
        }
      };
      // the products of a tile's fragments (FG filters x 16 windows) into S;
      // returns ||x^_w|| of the lane's window (fp32, rounded as stated above)
      auto products = [&](const uint2 (&A)[KS][QL], float4v (&S)[NT]) -> float {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) S[nt] = float4v{0.0f, 0.0f, 0.0f, 0.0f};
        float ss = 0.0f;
#pragma unroll
        for (int t = 0; t < KS; ++t) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) S[nt] = mfma_taps<KW>(rb[nt][t], A[t], S[nt]);
#pragma unroll
          for (int j = 0; j < QL; ++j) ss = sq2(A[t][j].y, sq2(A[t][j].x, ss));
        }
        ss += __shfl_xor(ss, 16, kWave);
        ss += __shfl_xor(ss, 32, kWave);
        return __builtin_sqrtf(ss);
      };
      // the signs of tile mt: one ballot per (filter block, element) gives
      // the 16-window fields of four filters at once
      auto extract = [&](int mt, const float4v (&S)[NT], float xn) {
        const uint64_t vmask = __builtin_amdgcn_ballot_w64(16 * mt + n16 < nb_item);
        uint64_t unt[NT][4];
        uint64_t any = 0;
        uint32_t mlo = 0, mhi = 0;  // lane 4 nt + i: the mask of (nt, i)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float sv = S[nt][i];
            const uint64_t tr = __builtin_amdgcn_ballot_w64(
                __builtin_fabsf(sv) > __builtin_fmaf(kk[nt][i].x, xn, kk[nt][i].y));
            const uint64_t pos = __builtin_amdgcn_ballot_w64(sv >= 0.0f);
            const uint64_t ones = tr & pos & vmask;
            unt[nt][i] = vmask & ~tr;
            any |= unt[nt][i];
            const bool mine = lane == 4 * nt + i;
            mlo = mine ? (uint32_t)ones : mlo;
            mhi = mine ? (uint32_t)(ones >> 32) : mhi;
          }
        }
        if (lane < 4 * NT)
          bm[w][lane >> 2][lane & 3][mt] = ((uint64_t)mhi << 32) | mlo;
        // untrusted pairs, appended in lane order (a full queue drops them
        // and the item goes down the exact path below)
        if (any) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint64_t u = unt[nt][i];
              if (u) {
                const int slot = qc + (int)__builtin_amdgcn_mbcnt_hi(
                                          (uint32_t)(u >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)u, 0u));
                if (((u >> lane) & 1ull) && slot < kQcapMulti) {
                  qwin[w][slot] = (uint8_t)(16 * mt + n16);
                  qfil[w][slot] = (uint8_t)(16 * nt + 4 * g + i);
                }
                qc += (int)__builtin_popcountll(u);
              }
            }
          }
        }
      };
      // tiles of 16 windows holding at least one window of the series, two in
      // flight: while tile mt's signs are read, tile mt + 1's products run and
      // tile mt + 2's fragments load
      const int ntile = (nwin + 15) / 16;
      float4v S0[NT], S1[NT];
      uint2 A0[KS][QL], A1[KS][QL];
      frags(0, A0);
      float x0 = products(A0, S0), x1 = 0.0f;
      if (1 < ntile) frags(1, A1);
      for (int mt = 0; mt < ntile; mt += 2) {
        if (mt + 1 < ntile) {
          x1 = products(A1, S1);
          if (mt + 2 < ntile) frags(mt + 2, A0);
        }
        extract(mt, S0, x0);
        if (mt + 1 < ntile) {
          if (mt + 2 < ntile) {
            x0 = products(A0, S0);
            if (mt + 3 < ntile) frags(mt + 3, A1);
          }
          extract(mt + 1, S1, x1);
        }
      }
      full = qc > kQcapMulti;
    }
    // tiles whose masks hold this item's signs (the others are read as 0)
    const int nfill = full ? kMtItem : (nwin + 15) / 16;
    wave_sync_lds();
    if (full) {
      // every (window, filter) pair of the item in float64, one per lane
      for (int i = lane; i < NT * 4 * kMtItem; i += kWave) (&bm[w][0][0][0])[i] = 0ull;
      wave_sync_lds();
      for (int pidx = lane; pidx < nwin * FG; pidx += kWave) {
        const int wl = pidx / FG, fl = pidx - wl * FG, r = fl & 15;
        if (exact_sign<W>(&xs[w][wl * D], rs[fl]))
          atomicOr(&bm[w][fl >> 4][r & 3][wl >> 4], 1ull << (16 * (r >> 2) + (wl & 15)));
      }
      repaired += (unsigned long long)(nwin * FG);
    } else if (qc > 0) {
      // the queued pairs in float64, one per lane
      for (int b = 0; b < qc; b += kWave) {
        if (b + lane < qc) {
          const int wl = qwin[w][b + lane], fl = qfil[w][b + lane], r = fl & 15;
          if (exact_sign<W>(&xs[w][wl * D], rs[fl]))
            atomicOr(&bm[w][fl >> 4][r & 3][wl >> 4], 1ull << (16 * (r >> 2) + (wl & 15)));
        }
      }
      repaired += (unsigned long long)qc;
    }
    wave_sync_lds();
    // the item's words of every filter's stream: 32-bit word j of filter
    // 16 nt + 4 g + i is field g of the masks of tiles 2 j and 2 j + 1
    const int nwords = (cur.nb + 63) / 64;
    for (int e = lane; e < FG * WPI; e += kWave) {
      const int fl = e / WPI, j = e - fl * WPI;
      const int64_t wd = (int64_t)cur.c * (kSubMulti / 64) + (j >> 1);
      if (wd < nwords) {
        const int nt = fl >> 4, r = fl & 15, gg = r >> 2, ii = r & 3;
        const uint64_t m0 = 2 * j < nfill ? bm[w][nt][ii][2 * j] : 0ull;
        const uint64_t m1 = 2 * j + 1 < nfill ? bm[w][nt][ii][2 * j + 1] : 0ull;
        const uint32_t word = (uint32_t)((m0 >> (16 * gg)) & 0xFFFFu) |
                              ((uint32_t)((m1 >> (16 * gg)) & 0xFFFFu) << 16);
        bits32[2 * ((int64_t)(ma.fbase + fl) * total_words + cur.wo + wd) + (j & 1)] = word;
      }
    }
    // the masks are rewritten by the next item only after this wave's reads
    wave_sync_lds();
    cur = nxt;
  }
  if (lane == 0 && repair_count && repaired) atomicAdd(repair_count, repaired);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline size_t al256m(size_t v) { return (v + 255) & ~(size_t)255; }

// Padded filter length of the workspace copy (a multiple of 32 covers both
// MFMA depths).
static inline int ws_wp(int W) { return (W + 31) / 32 * 32; }

size_t sketch_multi_workspace_bytes(int F, int W) {
  const size_t WP = (size_t)ws_wp(W);
  return al256m((size_t)F * WP * 4) + al256m((size_t)F * WP * 2) + al256m((size_t)F * 8);
}

bool sketch_multi_supported(int W, int delta) {
  return (W == 80 && delta == 3) || (W == 64 && delta == 4) || (W == 128 && delta == 4) ||
         (W == 30 && delta == 5);
}

// Item size and register budget per shape, from timing on MI355X: windows of
// (128, 4) fill 16-tile items at 3 waves per SIMD; the other shapes do best
// with 8-tile items (half the LDS, so more workgroups per CU), at 4 waves
// where the registers allow it.
template <int W, int D>
struct MultiTuning {
  static constexpr int MT = (W == 128 && D == 4) ? 16 : 8;
  static constexpr int WPE = (W == 128 && D == 4) || (W == 30 && D == 5) ? 3 : 4;
};

template <int W, int D, int KW, int NT>
static void launch_multi(const MultiArgs& ma, const float* x, const int64_t* x_off, int64_t N,
                         uint64_t* bits, int64_t total_words, const int64_t* bit_word_off,
                         int32_t* nbits, unsigned long long* rc, int* err, hipStream_t stream) {
  constexpr int MT = MultiTuning<W, D>::MT, WPE = MultiTuning<W, D>::WPE;
  const unsigned grid = resident_grid(
      reinterpret_cast<const void*>(&sketch_multi_kernel<W, D, KW, NT, MT, WPE>), N);
  sketch_multi_kernel<W, D, KW, NT, MT, WPE><<<grid, 256, 0, stream>>>(
      x, x_off, N, ma, bits, total_words, bit_word_off, nbits, rc, err);
}

template <int W, int D, int KW>
static void launch_group(const MultiArgs& ma, int nf, const float* x, const int64_t* x_off,
                         int64_t N, uint64_t* bits, int64_t total_words,
                         const int64_t* bit_word_off, int32_t* nbits, unsigned long long* rc,
                         int* err, hipStream_t stream) {
  if (nf >= 32)
    launch_multi<W, D, KW, 2>(ma, x, x_off, N, bits, total_words, bit_word_off, nbits, rc, err,
                              stream);
  else
    launch_multi<W, D, KW, 1>(ma, x, x_off, N, bits, total_words, bit_word_off, nbits, rc, err,
                              stream);
}

static void multi_layout(int F, int W, size_t& o_rh, size_t& o_kst) {
  const size_t WP = (size_t)ws_wp(W);
  o_rh = al256m((size_t)F * WP * 4);
  o_kst = o_rh + al256m((size_t)F * WP * 2);
}

static ssh_status multi_check(int F, int W, int delta) {
  if (!sketch_multi_supported(W, delta))
    return fail(SSH_EUNSUPPORTED, "ssh_sketch_multi: no matrix-core kernel for this (W, delta)");
  if (F < 16 || F > 64 || F % 16 != 0)
    return fail(SSH_EINVAL, "ssh_sketch_multi: F must be 16, 32, 48 or 64");
  return SSH_OK;
}

// Smallest fp16 value >= v (v positive, within fp16's normal range).
static uint16_t half_bits_up(double v) {
  uint16_t h = to_half_bits((float)v);
  if ((double)__builtin_bit_cast(_Float16, h) < v) ++h;  // next positive fp16
  return h;
}

// The filter block in `ws`: float32 rows and fp16 rows (zero-padded to a
// multiple of 32 taps), and each filter's margin constants
//     K1 = c1a ||c|| (1 + 2^-12),  K0 = (c0a + c1a 2^-14 sum c_k) (1 + 2^-12)
// (rounded up; c the margin weights, c1a and c0a the single-filter L1
// margin's constants for them).  Every filter passes the checks of the
// single-filter sketch.
ssh_status sketch_multi_prepare(const float* R, int F, int W, int delta, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
  ssh_status st = multi_check(F, W, delta);
  if (st != SSH_OK) return st;
  const size_t bytes = sketch_multi_workspace_bytes(F, W);
  if (ws_bytes < bytes) return fail(SSH_EINVAL, "ssh_sketch_multi_prepare: workspace too small");
  const int WP = ws_wp(W);
  size_t o_rh, o_kst;
  multi_layout(F, W, o_rh, o_kst);
  std::vector<unsigned char> host(bytes, 0);
  float* r32 = reinterpret_cast<float*>(host.data());
  uint16_t* rh = reinterpret_cast<uint16_t*>(host.data() + o_rh);
  float* kst = reinterpret_cast<float*>(host.data() + o_kst);
  const double v = 0x1p-11 / (1 - 0x1p-11);
  const double c_tiny =
      (double)__builtin_bit_cast(_Float16, half_bits_up(0x1p-14 * (1 + v) / (2 * v + v * v)));
  for (int f = 0; f < F; ++f) {
    FilterArgs fa;
    const float* r = R + (int64_t)f * W;
    st = make_filter_args(r, W, delta, fa);
    if (st != SSH_OK) return st;
    double l1c = 0.0, l2c = 0.0;
    for (int k = 0; k < W; ++k) {
      const float a = __builtin_fabsf(r[k]);
      const bool tiny = a != 0.0f && a < 0x1p-14f;
      r32[(size_t)f * WP + k] = r[k];
      rh[(size_t)f * WP + k] = tiny ? 0 : to_half_bits(r[k]);
      const double c = tiny ? c_tiny : __builtin_fabs((double)(_Float16)r[k]);
      l1c += c;
      l2c += c * c;
    }
    const double slack = 1 + 0x1p-12;
    kst[2 * f] = round_up_f32((double)fa.c1a * std::sqrt(l2c) * (1 + 0x1p-40) * slack);
    kst[2 * f + 1] =
        round_up_f32(((double)l1_margin_abs(l1c, W) + (double)fa.c1a * 0x1p-14 * l1c) * slack);
  }
  // the host copy is released on return: wait for the upload
  if (hipMemcpyAsync(ws, host.data(), bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_sketch_multi_prepare: filter upload failed");
  return SSH_OK;
}

ssh_status sketch_multi_launch(const float* x, const int64_t* x_off, int64_t N, const void* ws,
                               int F, int W, int delta, uint64_t* bits, int64_t total_words,
                               const int64_t* bit_word_off, int32_t* nbits,
                               uint64_t* repair_count, int kdepth, hipStream_t stream) {
  ssh_status st = multi_check(F, W, delta);
  if (st != SSH_OK) return st;
  if (kdepth != 0 && kdepth != 16 && kdepth != 32)
    return fail(SSH_EINVAL, "ssh_sketch_multi: kdepth must be 0, 16 or 32");
  if (N == 0) return SSH_OK;
  int* err = sketch_err_ptr();
  if (err == nullptr) return fail(SSH_EDEVICE, "ssh_sketch_multi: cannot resolve error flag");
  // 32 taps per instruction where the filter fills them; else 16 (W = 80 would
  // pad to 96 taps at 32)
  const int KW = kdepth != 0 ? kdepth : (W % 32 == 0 ? 32 : 16);
  size_t o_rh, o_kst;
  multi_layout(F, W, o_rh, o_kst);
  const unsigned char* base = static_cast<const unsigned char*>(ws);
  unsigned long long* rc = reinterpret_cast<unsigned long long*>(repair_count);
  for (int fb = 0; fb < F; fb += 32) {
    MultiArgs ma;
    ma.r32 = reinterpret_cast<const float*>(base);
    ma.rh = reinterpret_cast<const uint2*>(base + o_rh);
    ma.kst = reinterpret_cast<const float2*>(base + o_kst);
    ma.WP = ws_wp(W);
    ma.fbase = fb;
    const int nf = F - fb;
#define SSH_MULTI(WW, DD)                                                                        \
  if (W == WW && delta == DD) {                                                                  \
    if (KW == 16)                                                                                \
      launch_group<WW, DD, 16>(ma, nf, x, x_off, N, bits, total_words, bit_word_off, nbits, rc,  \
                               err, stream);                                                     \
    else                                                                                         \
      launch_group<WW, DD, 32>(ma, nf, x, x_off, N, bits, total_words, bit_word_off, nbits, rc,  \
                               err, stream);                                                     \
  }
    SSH_MULTI(80, 3)
    SSH_MULTI(64, 4)
    SSH_MULTI(128, 4)
    SSH_MULTI(30, 5)
#undef SSH_MULTI
    st = check_launch("ssh_sketch_multi");
    if (st != SSH_OK) return st;
  }
  return SSH_OK;
}

}  // namespace ssh
