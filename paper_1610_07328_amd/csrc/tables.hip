// Band keys and hash tables (Algorithm 1: every series goes into each of the
// L hash tables under one key per table).
//
// Keys: table l folds its K hash values with the SplitMix64 output function.
// Tables: the keys [N][L] are first transposed to table-major [L][N]; then,
// per table, a stable LSD radix sort of (key, id) on the top B bits of the
// key (table_sort_bits: 24 for N <= 2^24, else 32), B / 8 digit passes: the
// probe finds a bucket by the run of its top B bits, and 24 bits keep runs
// short at that size.  Each pass is four launches over all tables at
// once: per-tile digit histograms, a segmented reduce and then scan of the
// (digit, tile) counts, and a stable scatter.  The scatter ranks elements
// inside a wavefront with a ballot-based match of equal digits, keeps one
// running count per (wave, digit) in LDS, reorders the tile in LDS and writes
// each digit's run contiguously.  The histogram and scatter take their tiles
// in XCD-contiguous order, so the neighbouring partial lines that consecutive
// tiles write meet in one L2.
#include "band.hpp"

namespace ssh {

constexpr int kBkMaxK = 16;  // bands staged in LDS up to this K

// Item g = s L + l (series s, table l) folds hash values [g K, g K + K):
// with H = K L the bands of consecutive items are consecutive.  Each wave
// takes 64 items, loads their 64 K values with coalesced 8-byte loads into LDS
// and then folds one item per lane.
__global__ __launch_bounds__(256) void band_keys_kernel(const uint64_t* __restrict__ hv, int64_t N,
                                                        int K, int L, uint64_t seed,
                                                        uint64_t* __restrict__ keys) {
  __shared__ __attribute__((aligned(16))) uint64_t st[4][kWave * kBkMaxK];
  const int64_t total = N * (int64_t)L;
  const int H = K * L;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = lane_id();
  for (int64_t g0 = ((int64_t)blockIdx.x * 4 + w) * kWave; g0 < total;
       g0 += (int64_t)gridDim.x * 4 * kWave) {
    const int n_items = total - g0 < kWave ? (int)(total - g0) : kWave;
    const int nv = n_items * K;
    const uint64_t* src = hv + g0 * K;
    if ((((uintptr_t)src) & 15) == 0 && (nv & 1) == 0) {  // 16-byte loads of value pairs
      const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(src);
      ulonglong2* d2 = reinterpret_cast<ulonglong2*>(st[w]);
      for (int j = lane; j < nv / 2; j += kWave) d2[j] = s2[j];
    } else {
      for (int j = lane; j < nv; j += kWave) st[w][j] = src[j];
    }
    wave_sync_lds();
    if (lane < n_items) {
      const int64_t g = g0 + lane;
      const int64_t s = g / L;
      const int l = (int)(g - s * L);
      keys[g] = hv[s * H] == SSH_HV_EMPTY ? SSH_KEY_EMPTY : band_fold(&st[w][lane * K], K, l, seed);
    }
    wave_sync_lds();
  }
}

// K > kBkMaxK: one thread per item, straight from global memory
__global__ __launch_bounds__(256) void band_keys_wide_kernel(const uint64_t* __restrict__ hv,
                                                             int64_t N, int K, int L, uint64_t seed,
                                                             uint64_t* __restrict__ keys) {
  const int64_t total = N * (int64_t)L;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int H = K * L;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t s = g / L;
    const int l = (int)(g - s * L);
    keys[g] = hv[s * H] == SSH_HV_EMPTY ? SSH_KEY_EMPTY : band_fold(hv + g * K, K, l, seed);
  }
}

ssh_status band_keys_launch(const uint64_t* hv, int64_t N, int K, int L, uint64_t seed,
                            uint64_t* keys, hipStream_t stream) {
  if (N == 0) return SSH_OK;
  if (K <= kBkMaxK)
    band_keys_kernel<<<grid_for(N * (int64_t)L, 256, 1 << 16), 256, 0, stream>>>(hv, N, K, L, seed,
                                                                                keys);
  else
    band_keys_wide_kernel<<<grid_for(N * (int64_t)L, 256, 1 << 16), 256, 0, stream>>>(hv, N, K, L,
                                                                                     seed, keys);
  return check_launch("ssh_band_keys");
}

// ---------------------------------------------------------------------------
// radix sort of (key, id) per table on key bits [32, 64)
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;  // 2048: a 30 KB LDS tile, five workgroups per CU
constexpr int kRsWaves = kRsThreads / kWave;
constexpr int kRsPerWave = kWave * kRsItems;   // 512 contiguous elements per wave

struct RsIn {
  const uint64_t* keys;  // series-major [N * L] when sm, else table-major [L * N]
  const uint32_t* ids;   // null on pass 0 (ids are the series index)
  bool first;
  bool sm;
};

__device__ __forceinline__ void rs_load(const RsIn in, int64_t e, int64_t N, int L, int l,
                                        uint64_t& key, uint32_t& id) {
  if (in.first) {
    key = in.sm ? in.keys[e * L + l] : in.keys[(int64_t)l * N + e];
    id = (uint32_t)e;
  } else {
    key = in.keys[(int64_t)l * N + e];
    id = in.ids[(int64_t)l * N + e];
  }
}

// (table l, tile b) of this workgroup in a (nblk, L) grid, taken in
// XCD-contiguous order (xcd_linear_block), so that what consecutive tiles
// write next to each other (count columns, digit runs) goes through one L2.
__device__ __forceinline__ void xcd_tile(int nblk, int& l, int& b) {
  const int64_t v = xcd_linear_block();
  l = (int)(v / nblk);
  b = (int)(v - (int64_t)l * nblk);
}

__global__ __launch_bounds__(kRsThreads) void rs_hist_kernel(RsIn in, int64_t N, int L, int shift,
                                                             int nblk, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  int l, b;
  xcd_tile(nblk, l, b);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)b * kRsTile;
  for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) {
    const int64_t e = base + i;
    if (e < N) {
      uint64_t key;
      uint32_t id;
      rs_load(in, e, N, L, l, key, id);
      atomicAdd(&h[(key >> shift) & 255], 1u);
    }
  }
  __syncthreads();
  hist[((int64_t)l * 256 + threadIdx.x) * nblk + b] = h[threadIdx.x];
}

// Exclusive scan, per table, of the n = 256 * nblk counts in (digit, tile)
// order, in S segments of `seg` counts (seg a multiple of 4): rs_reduce sums
// each segment; rs_scan adds the sums of the segments before its own and
// scans its segment in tiles of 1024 counts (four per thread).
__global__ __launch_bounds__(kRsThreads) void rs_reduce_kernel(const uint32_t* __restrict__ hist,
                                                               int64_t n, int64_t seg,
                                                               uint32_t* __restrict__ seg_sum) {
  __shared__ uint32_t ws[kRsWaves];
  const int l = blockIdx.y, sg = blockIdx.x;
  const uint32_t* h = hist + (int64_t)l * n;
  const int64_t lo = (int64_t)sg * seg;
  const int64_t hi = lo + seg < n ? lo + seg : n;
  uint32_t sum = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kRsThreads) sum += h[i];
  sum = wave_sum(sum);
  if (lane_id() == 0) ws[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int i = 0; i < kRsWaves; ++i) t += ws[i];
    seg_sum[(int64_t)l * gridDim.x + sg] = t;
  }
}

__global__ __launch_bounds__(kRsThreads) void rs_scan_kernel(uint32_t* __restrict__ hist, int64_t n,
                                                             int64_t seg,
                                                             const uint32_t* __restrict__ seg_sum) {
  __shared__ uint32_t wtot[kRsWaves];
  __shared__ uint32_t carry_s;
  const int l = blockIdx.y, sg = blockIdx.x;
  const int w = threadIdx.x / kWave;
  uint32_t* h = hist + (int64_t)l * n;
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int i = 0; i < sg; ++i) c += seg_sum[(int64_t)l * gridDim.x + i];
    carry_s = c;
  }
  __syncthreads();
  uint32_t carry = carry_s;
  const int64_t lo = (int64_t)sg * seg;
  const int64_t hi = lo + seg < n ? lo + seg : n;
  for (int64_t t0 = lo; t0 < hi; t0 += 4 * kRsThreads) {
    const int64_t i = t0 + 4 * threadIdx.x;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i + 3 < hi) {
      v = *reinterpret_cast<const uint4*>(h + i);
    } else {
      if (i < hi) v.x = h[i];
      if (i + 1 < hi) v.y = h[i + 1];
      if (i + 2 < hi) v.z = h[i + 2];
    }
    const uint32_t tsum = v.x + v.y + v.z + v.w;
    const uint32_t incl = wave_incl_scan(tsum);
    if (lane_id() == kWave - 1) wtot[w] = incl;
    __syncthreads();
    uint32_t before = carry;
    for (int ww = 0; ww < w; ++ww) before += wtot[ww];
    uint32_t tile = 0;
    for (int ww = 0; ww < kRsWaves; ++ww) tile += wtot[ww];
    uint32_t run = before + incl - tsum;
    const uint4 o = make_uint4(run, run + v.x, run + v.x + v.y, run + v.x + v.y + v.z);
    if (i + 3 < hi) {
      *reinterpret_cast<uint4*>(h + i) = o;
    } else {
      if (i < hi) h[i] = o.x;
      if (i + 1 < hi) h[i + 1] = o.y;
      if (i + 2 < hi) h[i + 2] = o.z;
    }
    carry += tile;
    __syncthreads();  // wtot is reused by the next tile
  }
}

__global__ __launch_bounds__(kRsThreads) void rs_scatter_kernel(RsIn in, int64_t N, int L,
                                                                int shift, int nblk,
                                                                const uint32_t* __restrict__ offs,
                                                                uint64_t* __restrict__ out_keys,
                                                                uint32_t* __restrict__ out_ids) {
  __shared__ uint32_t wcnt[kRsWaves][256];
  __shared__ uint32_t tstart[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint64_t skeys[kRsTile];
  __shared__ uint32_t sids[kRsTile];
  int l, b;
  xcd_tile(nblk, l, b);
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const int64_t tbase = (int64_t)b * kRsTile;
  const int64_t wbase = tbase + (int64_t)w * kRsPerWave;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t key[kRsItems];
  uint32_t id[kRsItems];
  uint32_t rank[kRsItems];
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) {
    const int64_t e = wbase + q * kWave + lane;
    const bool valid = e < N;
    key[q] = 0;
    id[q] = 0;
    if (valid) rs_load(in, e, N, L, l, key[q], id[q]);
    const uint32_t d = (uint32_t)(key[q] >> shift) & 255u;
    uint64_t peers = ballot64(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bal = ballot64(valid && on);
      peers &= on ? bal : ~bal;
    }
    rank[q] = 0;
    if (valid) {
      const uint32_t before = wcnt[w][d];
      rank[q] = before + (uint32_t)__builtin_popcountll(peers & lt_mask);
      if ((peers & lt_mask) == 0) wcnt[w][d] = before + (uint32_t)__builtin_popcountll(peers);
    }
    wave_sync_lds();
  }
  __syncthreads();
  // per digit: exclusive offsets over waves, tile totals, tile-local starts
  {
    const int d = threadIdx.x;  // 256 threads, one digit each
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) {
      const uint32_t c = wcnt[ww][d];
      wcnt[ww][d] = run;
      run += c;
    }
    tstart[d] = run;  // tile total for now
    gbase[d] = offs[((int64_t)l * 256 + d) * nblk + b];
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    // exclusive scan of the 256 tile totals by one wave (4 per lane)
    const int t = threadIdx.x;
    uint32_t v0 = tstart[4 * t], v1 = tstart[4 * t + 1], v2 = tstart[4 * t + 2], v3 = tstart[4 * t + 3];
    const uint32_t tot = v0 + v1 + v2 + v3;
    const uint32_t incl = wave_incl_scan(tot);
    uint32_t run = incl - tot;
    tstart[4 * t] = run;
    run += v0;
    tstart[4 * t + 1] = run;
    run += v1;
    tstart[4 * t + 2] = run;
    run += v2;
    tstart[4 * t + 3] = run;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) {
    const int64_t e = wbase + q * kWave + lane;
    if (e < N) {
      const uint32_t d = (uint32_t)(key[q] >> shift) & 255u;
      const uint32_t pos = tstart[d] + wcnt[w][d] + rank[q];
      skeys[pos] = key[q];
      sids[pos] = id[q];
    }
  }
  __syncthreads();
  const int64_t left = N - tbase;
  const int cnt = left < kRsTile ? (int)left : kRsTile;
  for (int p = threadIdx.x; p < cnt; p += kRsThreads) {
    const uint64_t k = skeys[p];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const int64_t dst = (int64_t)gbase[d] + (p - (int64_t)tstart[d]);
    out_keys[(int64_t)l * N + dst] = k;
    out_ids[(int64_t)l * N + dst] = sids[p];
  }
}

// keys [N][L] -> out [L][N] through an LDS tile of kTrRows series, so both
// the reads and the writes are contiguous (L <= kTrMaxL)
constexpr int kTrRows = 64;
constexpr int kTrMaxL = 64;

__global__ __launch_bounds__(256) void keys_transpose_kernel(const uint64_t* __restrict__ keys,
                                                             int64_t N, int L,
                                                             uint64_t* __restrict__ out) {
  __shared__ uint64_t tile[kTrRows * kTrMaxL];
  const int64_t s0 = (int64_t)blockIdx.x * kTrRows;
  const int rows = N - s0 < kTrRows ? (int)(N - s0) : kTrRows;
  const int n = rows * L;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tile[i] = keys[s0 * L + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int l = i / rows, r = i - l * rows;
    out[(int64_t)l * N + s0 + r] = tile[r * L + l];
  }
}

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kRsMaxSeg = 64;  // scan segments per table

size_t table_workspace_bytes(int64_t N, int L) {
  const int64_t nblk = ceil_div(N > 0 ? N : 1, kRsTile);
  return align256((size_t)N * L * 8) + align256((size_t)N * L * 4) +
         align256((size_t)L * 256 * nblk * 4) + align256((size_t)L * kRsMaxSeg * 4);
}

ssh_status table_build_launch(const uint64_t* keys, int64_t N, int L, uint64_t* tab_keys,
                              uint32_t* tab_ids, void* ws, size_t ws_bytes, hipStream_t stream,
                              int sort_bits) {
  if (N == 0) return SSH_OK;
  if (ws_bytes < table_workspace_bytes(N, L))
    return fail(SSH_EINVAL, "ssh_table_build: workspace too small");
  const int nblk = (int)ceil_div(N, kRsTile);
  unsigned char* p = reinterpret_cast<unsigned char*>(ws);
  uint64_t* alt_keys = reinterpret_cast<uint64_t*>(p);
  p += align256((size_t)N * L * 8);
  uint32_t* alt_ids = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)N * L * 4);
  uint32_t* hist = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)L * 256 * nblk * 4);
  uint32_t* seg_sum = reinterpret_cast<uint32_t*>(p);
  const dim3 grid(nblk, L);
  // scan segments: about 4096 counts each, a multiple of 4, at most kRsMaxSeg
  const int64_t n = (int64_t)256 * nblk;
  int nseg = (int)ceil_div(n, 4096);
  if (nseg > kRsMaxSeg) nseg = kRsMaxSeg;
  const int64_t seg = (ceil_div(n, nseg) + 3) & ~(int64_t)3;
  nseg = (int)ceil_div(n, seg);
  const dim3 sgrid(nseg, L);
  // The passes alternate between the output (tab) and the workspace (alt),
  // the last one writing tab.  With L <= kTrMaxL the keys are first
  // transposed into the buffer pass 0 does not write, so every pass reads
  // table-major; otherwise pass 0 reads the series-major keys.
  const int passes = (sort_bits > 0 ? sort_bits : table_sort_bits(N)) / 8;
  auto to_tab = [&](int pass) { return (passes - 1 - pass) % 2 == 0; };
  const bool transposed = L <= kTrMaxL;
  uint64_t* tr = to_tab(0) ? alt_keys : tab_keys;
  if (transposed)
    keys_transpose_kernel<<<(unsigned)ceil_div(N, kTrRows), 256, 0, stream>>>(keys, N, L, tr);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 64 - 8 * passes + 8 * pass;
    RsIn in;
    if (pass == 0)
      in = transposed ? RsIn{tr, nullptr, true, false} : RsIn{keys, nullptr, true, true};
    else if (to_tab(pass))
      in = RsIn{alt_keys, alt_ids, false, false};
    else
      in = RsIn{tab_keys, tab_ids, false, false};
    uint64_t* ok = to_tab(pass) ? tab_keys : alt_keys;
    uint32_t* oi = to_tab(pass) ? tab_ids : alt_ids;
    rs_hist_kernel<<<grid, kRsThreads, 0, stream>>>(in, N, L, shift, nblk, hist);
    rs_reduce_kernel<<<sgrid, kRsThreads, 0, stream>>>(hist, n, seg, seg_sum);
    rs_scan_kernel<<<sgrid, kRsThreads, 0, stream>>>(hist, n, seg, seg_sum);
    rs_scatter_kernel<<<grid, kRsThreads, 0, stream>>>(in, N, L, shift, nblk, hist, ok, oi);
  }
  return check_launch("ssh_table_build");
}

// ---------------------------------------------------------------------------
// Updates of built tables (Algorithm 1's tables, kept and updated: Section 1,
// data-independent hashing lets new series join without touching the others).
// ---------------------------------------------------------------------------
__device__ int g_table_err;

int take_table_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_table_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_table_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

// Entries of sorted run t (n entries) whose top bits are below (strict) or
// at most (!strict) v.
__device__ __forceinline__ int64_t count_below(const uint64_t* __restrict__ t, int64_t n, int sh,
                                               uint64_t v, bool strict) {
  int64_t a = 0, b = n;
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    const uint64_t u = t[mid] >> sh;
    if (strict ? u < v : u <= v) a = mid + 1;
    else b = mid;
  }
  return a;
}

// Merge of table l's N old entries (A) and M new ones (B, ids 0..M-1 standing
// for id_base..id_base+M-1, above every old id), both ordered by top bits
// with ids ascending: an old entry
// goes after the new ones with smaller top bits, a new one after the old ones
// with smaller or equal top bits (all old ids are smaller), which is the order
// a build over the N + M series gives.
__global__ __launch_bounds__(256) void table_merge_kernel(
    const uint64_t* __restrict__ a_keys, const uint32_t* __restrict__ a_ids, int64_t N,
    const uint64_t* __restrict__ b_keys, const uint32_t* __restrict__ b_ids, int64_t M, int L,
    int64_t id_base, int sh, uint64_t* __restrict__ out_keys, uint32_t* __restrict__ out_ids) {
  const int64_t T = N + M;
  const int64_t per = (T + 255) / 256 * 256;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < per * L;
       g += (int64_t)gridDim.x * 256) {
    const int l = (int)(g / per);
    const int64_t e = g - (int64_t)l * per;
    if (e >= T) continue;
    const uint64_t* ak = a_keys + (int64_t)l * N;
    const uint64_t* bk = b_keys + (int64_t)l * M;
    uint64_t key;
    uint32_t id;
    int64_t pos;
    if (e < N) {
      key = ak[e];
      id = a_ids[(int64_t)l * N + e];
      pos = e + count_below(bk, M, sh, key >> sh, true);
    } else {
      const int64_t j = e - N;
      key = bk[j];
      id = (uint32_t)(id_base + b_ids[(int64_t)l * M + j]);
      pos = j + count_below(ak, N, sh, key >> sh, false);
    }
    out_keys[(int64_t)l * T + pos] = key;
    out_ids[(int64_t)l * T + pos] = id;
  }
}

size_t table_insert_workspace_bytes(int64_t M, int L) {
  return align256((size_t)M * L * 8) + align256((size_t)M * L * 4) + table_workspace_bytes(M, L);
}

ssh_status table_insert_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N,
                               const uint64_t* new_keys, int64_t M, int L, int64_t id_base,
                               uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (N > 0 && table_sort_bits(N) != table_sort_bits(N + M))
    return fail(SSH_EUNSUPPORTED, "ssh_table_insert: the sort width changes at 2^24 series; "
                                  "build the tables again");
  if (ws_bytes < table_insert_workspace_bytes(M, L))
    return fail(SSH_EINVAL, "ssh_table_insert: workspace too small");
  if (N + M == 0) return SSH_OK;
  const int B = table_sort_bits(N + M);
  unsigned char* p = reinterpret_cast<unsigned char*>(ws);
  uint64_t* bk = reinterpret_cast<uint64_t*>(p);
  p += align256((size_t)M * L * 8);
  uint32_t* bi = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)M * L * 4);
  if (M > 0) {
    const ssh_status st = table_build_launch(new_keys, M, L, bk, bi, p, table_workspace_bytes(M, L),
                                             stream, B);
    if (st != SSH_OK) return st;
  }
  const int64_t total = ceil_div(N + M, 256) * 256 * L;
  table_merge_kernel<<<grid_for(total, 256, 1 << 16), 256, 0, stream>>>(
      tab_keys, tab_ids, N, bk, bi, M, L, id_base, 64 - B, out_keys, out_ids);
  return check_launch("ssh_table_insert");
}

// Deletion: table l keeps, in order, its entries whose id is not marked dead.
// Per (table, tile of kRsTile entries) live counts, then per table a scan
// (which checks that n_live entries survive), then a stable scatter.
__global__ __launch_bounds__(256) void table_live_count_kernel(
    const uint32_t* __restrict__ ids, int64_t N, int L, const uint8_t* __restrict__ dead,
    int64_t id_bound, int nblk, uint32_t* __restrict__ cnt, int* err) {
  __shared__ uint32_t c;
  const int l = blockIdx.y, b = blockIdx.x;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int i = threadIdx.x; i < kRsTile; i += 256) {
    const int64_t e = (int64_t)b * kRsTile + i;
    if (e < N) {
      const uint32_t id = ids[(int64_t)l * N + e];
      if (id >= id_bound) atomicOr(err, 1);
      else mine += dead[id] == 0;
    }
  }
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) cnt[(int64_t)l * nblk + b] = c;
}

__global__ __launch_bounds__(256) void table_live_scan_kernel(uint32_t* __restrict__ cnt, int nblk,
                                                              int64_t n_live, int* err) {
  __shared__ uint32_t wsum[256 / kWave];
  __shared__ int64_t carry;
  const int l = blockIdx.x;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint32_t* c = cnt + (int64_t)l * nblk;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nblk; b0 += 256) {
    const int b = b0 + threadIdx.x;
    const uint32_t v = b < nblk ? c[b] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < 256 / kWave; ++i) {
      before += i < w ? wsum[i] : 0u;
      tot += wsum[i];
    }
    if (b < nblk) c[b] = (uint32_t)(carry + before + incl - v);
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && carry != n_live) atomicOr(err, 2);
}

__global__ __launch_bounds__(256) void table_live_scatter_kernel(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ids, int64_t N, int L,
    const uint8_t* __restrict__ dead, int64_t id_bound, int nblk, const uint32_t* __restrict__ off,
    int64_t n_live, uint64_t* __restrict__ out_keys, uint32_t* __restrict__ out_ids) {
  __shared__ uint32_t wc[256 / kWave];
  __shared__ uint32_t run;
  const int l = blockIdx.y, b = blockIdx.x;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) run = off[(int64_t)l * nblk + b];
  __syncthreads();
  for (int i0 = 0; i0 < kRsTile; i0 += 256) {
    const int64_t e = (int64_t)b * kRsTile + i0 + threadIdx.x;
    bool live = false;
    uint64_t key = 0;
    uint32_t id = 0;
    if (e < N) {
      id = ids[(int64_t)l * N + e];
      key = keys[(int64_t)l * N + e];
      live = id < id_bound && dead[id] == 0;
    }
    const uint64_t m = ballot64(live);
    if (lane == 0) wc[w] = (uint32_t)__builtin_popcountll(m);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < 256 / kWave; ++i) {
      before += i < w ? wc[i] : 0u;
      tot += wc[i];
    }
    const uint32_t rank = (uint32_t)__builtin_popcountll(m & ((1ull << lane) - 1ull));
    const int64_t dst = (int64_t)run + before + rank;
    if (live && dst < n_live) {
      out_keys[(int64_t)l * n_live + dst] = key;
      out_ids[(int64_t)l * n_live + dst] = id;
    }
    __syncthreads();
    if (threadIdx.x == 0) run += tot;
    __syncthreads();
  }
}

size_t table_delete_workspace_bytes(int64_t N, int L) {
  return align256((size_t)L * ceil_div(N > 0 ? N : 1, kRsTile) * 4);
}

ssh_status table_delete_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int L,
                               const uint8_t* dead, int64_t id_bound, int64_t n_live,
                               uint64_t* out_keys, uint32_t* out_ids, void* ws, size_t ws_bytes,
                               hipStream_t stream) {
  if (n_live > 0 && table_sort_bits(N) != table_sort_bits(n_live))
    return fail(SSH_EUNSUPPORTED, "ssh_table_delete: the sort width changes at 2^24 series; "
                                  "build the tables again");
  if (ws_bytes < table_delete_workspace_bytes(N, L))
    return fail(SSH_EINVAL, "ssh_table_delete: workspace too small");
  if (N == 0 || n_live == 0) return SSH_OK;
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_table_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_table_delete: cannot resolve error flag");
  const int nblk = (int)ceil_div(N, kRsTile);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(ws);
  const dim3 grid(nblk, L);
  table_live_count_kernel<<<grid, 256, 0, stream>>>(tab_ids, N, L, dead, id_bound, nblk, cnt, err);
  table_live_scan_kernel<<<L, 256, 0, stream>>>(cnt, nblk, n_live, err);
  table_live_scatter_kernel<<<grid, 256, 0, stream>>>(tab_keys, tab_ids, N, L, dead, id_bound, nblk,
                                                      cnt, n_live, out_keys, out_ids);
  return check_launch("ssh_table_delete");
}

}  // namespace ssh
