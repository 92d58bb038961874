// Query probe (Algorithm 2: the retrieved set R is the union, over the hash
// tables, of the query's bucket in each), then ranking of R.
//
// Three launches:
//  1. runs: one wavefront per query.  Per table, two searches (lanes 0-31 the
//     start, lanes 32-63 the end) find the run of entries whose top key bits
//     (the bits the tables are sorted on) equal the query's; the runs of all
//     tables, concatenated, are the
//     query's G entries.  Entries of a run with the query's full key are the
//     bucket.
//  2. parts: the G entries of a query are cut into F contiguous slices, one
//     workgroup each.  A member X of R is counted once, at the first table
//     whose key matches (X's keys in earlier tables are compared with the
//     query's), so no de-duplication structure is needed; its score is the
//     number of hash values it shares with the query.  Each part keeps its
//     first min(|R_f|, C) members by (score desc, id asc), through the
//     composite key (H - score) << 32 | id: a histogram of scores finds the
//     score level holding the C-th member, members above it are kept, and
//     among that level the smallest ids are taken (sorted in LDS when they
//     fit, else by a radix select over id bytes).
//  3. merge: one workgroup per query sorts the F parts' keys (bitonic, in LDS)
//     and keeps the first C.  The first C of R are among the parts' first C
//     (a member preceded by fewer than C members of R is preceded by fewer
//     than C members of its own part).
#include "common.hpp"

namespace ssh {

constexpr int kPrThreads = 256;
constexpr int kMaxL = 64;
constexpr int kMaxH = 1024;
constexpr int kTieCap = 1024;     // tied ids of one part sorted in LDS; more take the radix select
// Entries of one part whose scores are kept in LDS (32 KB).  A larger part
// scores its members again in every pass over them, so the cap covers the
// parts of queries whose buckets sum to about 130,000 entries.
constexpr int kScoreCap = 16384;
constexpr int kMergeCap = 4096;   // keys one merge sorts in LDS
constexpr int kMaxParts = 8;
constexpr uint16_t kNotMember = 0xFFFFu;

struct ProbeCtx {
  const uint64_t* tab_keys;
  const uint32_t* tab_ids;
  int64_t N;
  int L;
  const uint64_t* db_keys;
  const uint64_t* db_hv;
  int H;
};

__host__ __device__ inline int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Parts per query: as many as keep a merge within kMergeCap keys, at most kMaxParts.
__host__ __device__ inline int probe_parts(int C) {
  const int f = kMergeCap / pow2_at_least(C);
  return f < 1 ? 1 : (f > kMaxParts ? kMaxParts : f);
}

// Workspace: runs (glo [nq][L], gpre [nq][L + 1]) and parts (keys
// [nq][F][C], counts [nq][F], |R_f| [nq][F]).
struct ProbeWs {
  int64_t* glo;
  int64_t* gpre;
  uint64_t* keys;
  int64_t* rpart;
  uint32_t* nkeys;
};

__host__ __device__ inline size_t probe_ws_bytes(int nq, int L, int C) {
  const size_t F = (size_t)probe_parts(C);
  return (size_t)nq * L * 8 + (size_t)nq * (L + 1) * 8 + (size_t)nq * F * C * 8 +
         (size_t)nq * F * 8 + (((size_t)nq * F * 4 + 7) & ~(size_t)7);
}

__host__ __device__ inline ProbeWs probe_ws(void* ws, int nq, int L, int C) {
  const size_t F = (size_t)probe_parts(C);
  char* p = static_cast<char*>(ws);
  ProbeWs w;
  w.glo = reinterpret_cast<int64_t*>(p);
  p += (size_t)nq * L * 8;
  w.gpre = reinterpret_cast<int64_t*>(p);
  p += (size_t)nq * (L + 1) * 8;
  w.keys = reinterpret_cast<uint64_t*>(p);
  p += (size_t)nq * F * C * 8;
  w.rpart = reinterpret_cast<int64_t*>(p);
  p += (size_t)nq * F * 8;
  w.nkeys = reinterpret_cast<uint32_t*>(p);
  return w;
}

// ---------------------------------------------------------------------------
// 1. runs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void probe_runs_kernel(ProbeCtx c,
                                                           const uint64_t* __restrict__ q_keys,
                                                           ProbeWs ws) {
  __shared__ int64_t len[kMaxL];
  const int q = blockIdx.x;
  const int lane = lane_id();
  const int half = lane >> 5, t = lane & 31;
  const uint64_t* qk = q_keys + (int64_t)q * c.L;
  const bool empty = qk[0] == SSH_KEY_EMPTY || c.N == 0;
  for (int l0 = 0; l0 < c.L; l0 += 32) {
    const int l = l0 + t;
    int64_t bound = 0;
    if (l < c.L && !empty) {
      // half 0: first entry whose top bits are >= the query's; half 1: first >
      const uint64_t* tk = c.tab_keys + (int64_t)l * c.N;
      const int sh = 64 - table_sort_bits(c.N);
      const uint64_t hi = qk[l] >> sh;
      int64_t a = 0, b = c.N;
      while (a < b) {
        const int64_t mid = (a + b) >> 1;
        const uint64_t v = tk[mid] >> sh;
        if (half == 0 ? v < hi : v <= hi) a = mid + 1;
        else b = mid;
      }
      bound = a;
    }
    const int64_t end = __shfl_down(bound, 32, kWave);  // half 1's bound of the same table
    if (half == 0 && l < c.L) {
      ws.glo[(int64_t)q * c.L + l] = bound;
      len[l] = end - bound;
    }
  }
  wave_sync_lds();
  if (lane == 0) {
    int64_t* gpre = ws.gpre + (int64_t)q * (c.L + 1);
    int64_t s = 0;
    gpre[0] = 0;
    for (int l = 0; l < c.L; ++l) {
      s += len[l];
      gpre[l + 1] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// 2. parts
// ---------------------------------------------------------------------------
// Number of the H hash values of X equal to the query's (qh in LDS): the
// row is read 16 bytes at a time, sixteen loads in flight.
__device__ __forceinline__ int member_score(const ProbeCtx& c, uint32_t X, const uint64_t* qh) {
  const uint64_t* xh = c.db_hv + (int64_t)X * c.H;
  int score = 0;
  int j = 0;
  if ((c.H & 1) == 0 && ((uintptr_t)c.db_hv & 15) == 0) {  // rows are 16-byte aligned
    const ulonglong2* x2 = reinterpret_cast<const ulonglong2*>(xh);
    for (; j + 32 <= c.H; j += 32) {
      ulonglong2 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = x2[j / 2 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) score += (v[u].x == qh[j + 2 * u]) + (v[u].y == qh[j + 2 * u + 1]);
    }
    for (; j + 2 <= c.H; j += 2) {
      const ulonglong2 v = x2[j / 2];
      score += (v.x == qh[j]) + (v.y == qh[j + 1]);
    }
  }
  for (; j < c.H; ++j) score += xh[j] == qh[j];
  return score;
}

// Entry e of the concatenated key runs: the member it names, or -1 when its
// full key differs from the query's or the member already matched an earlier
// table (a member of R is counted at the first table whose key matches).
__device__ __forceinline__ int64_t entry_member(const ProbeCtx& c, const uint64_t* qk,
                                                const int64_t* glo, const int64_t* gpre,
                                                int64_t e) {
  int l = 0;
  while (l + 1 < c.L && gpre[l + 1] <= e) ++l;
  const int64_t idx = (int64_t)l * c.N + glo[l] + (e - gpre[l]);
  // the entry's key and id together; then the member's keys of the earlier
  // tables, all loads issued before any comparison
  const uint64_t key = c.tab_keys[idx];
  const uint32_t X = c.tab_ids[idx];
  if (key != qk[l]) return -1;
  const uint64_t* xk = c.db_keys + (int64_t)X * c.L;
  constexpr int kBatch = 8;
  for (int l0 = 0; l0 < l; l0 += kBatch) {
    uint64_t v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = l0 + u < l ? xk[l0 + u] : ~qk[l0 + u < l ? l0 + u : 0];
    bool seen = false;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) seen |= l0 + u < l && v[u] == qk[l0 + u < l ? l0 + u : 0];
    if (seen) return -1;
  }
  return X;
}

// Visit every member of R among entries [e0, e1) (once each) with its score.
// With `sc` set, the first visit records every entry's score (kNotMember for
// non-members) and later visits read it, reading the member's id only when
// need(score) holds.
template <typename F, typename Need>
__device__ __forceinline__ void for_members(const ProbeCtx& c, const uint64_t* qk, const uint64_t* qh,
                                            const int64_t* glo, const int64_t* gpre, int64_t e0,
                                            int64_t e1, uint16_t* sc, bool first, F&& f,
                                            Need&& need) {
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kPrThreads) {
    if (sc && !first) {
      const uint16_t v = sc[e - e0];
      if (v == kNotMember || !need((int)v)) continue;
      int l = 0;
      while (l + 1 < c.L && gpre[l + 1] <= e) ++l;
      const uint32_t X = c.tab_ids[(int64_t)l * c.N + glo[l] + (e - gpre[l])];
      f(X, (int)v);
      continue;
    }
    const int64_t X = entry_member(c, qk, glo, gpre, e);
    if (X < 0) {
      if (sc) sc[e - e0] = kNotMember;
      continue;
    }
    const int score = member_score(c, (uint32_t)X, qh);
    if (sc) sc[e - e0] = (uint16_t)score;
    f((uint32_t)X, score);
  }
}

template <typename T>
__device__ void bitonic_sort(T* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += kPrThreads) {
        const int p = i ^ j;
        if (p > i) {
          const T x = a[i], y = a[p];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kPrThreads) void probe_part_kernel(ProbeCtx c,
                                                                const uint64_t* __restrict__ q_keys,
                                                                const uint64_t* __restrict__ q_hv,
                                                                int C, int F, ProbeWs ws) {
  __shared__ uint64_t qk[kMaxL];
  __shared__ int64_t glo[kMaxL];
  __shared__ int64_t gpre[kMaxL + 1];
  __shared__ uint32_t bhist[256];
  __shared__ uint32_t ties[kTieCap];
  __shared__ uint16_t sc_buf[kScoreCap];
  __shared__ uint32_t nR, nsel, ntie;
  __shared__ int s_thr;
  __shared__ uint32_t prefix, need;
  // sized at launch: query hash values [H], score histogram [H + 1] (to 8
  // bytes), the part's selection [C]
  extern __shared__ __attribute__((aligned(16))) uint64_t pdyn[];
  uint64_t* qh = pdyn;
  uint32_t* hist = reinterpret_cast<uint32_t*>(pdyn + c.H);
  uint64_t* sel = pdyn + c.H + (c.H + 2) / 2;

  const int q = blockIdx.x / F;
  const int part = blockIdx.x - q * F;
  const int tid = threadIdx.x;
  const int64_t* wgpre = ws.gpre + (int64_t)q * (c.L + 1);
  const int64_t G = wgpre[c.L];
  const int64_t e0 = G * part / F, e1 = G * (part + 1) / F;
  uint64_t* out = ws.keys + ((int64_t)q * F + part) * C;
  if (e0 == e1) {  // nothing in this part (a query without shingles has no entries)
    if (tid == 0) {
      ws.nkeys[(int64_t)q * F + part] = 0;
      ws.rpart[(int64_t)q * F + part] = 0;
    }
    return;
  }
  for (int i = tid; i < c.L; i += kPrThreads) {
    qk[i] = q_keys[(int64_t)q * c.L + i];
    glo[i] = ws.glo[(int64_t)q * c.L + i];
  }
  for (int i = tid; i <= c.L; i += kPrThreads) gpre[i] = wgpre[i];
  for (int i = tid; i < c.H; i += kPrThreads) qh[i] = q_hv[(int64_t)q * c.H + i];
  for (int i = tid; i <= c.H; i += kPrThreads) hist[i] = 0;
  if (tid == 0) {
    nR = 0;
    nsel = 0;
    ntie = 0;
  }
  __syncthreads();
  uint16_t* sc = e1 - e0 <= kScoreCap ? sc_buf : nullptr;
  auto all = [](int) { return true; };
  // score histogram over the part's members
  for_members(c, qk, qh, glo, gpre, e0, e1, sc, true, [&](uint32_t X, int score) {
    (void)X;
    atomicAdd(&hist[score], 1u);
    atomicAdd(&nR, 1u);
  }, all);
  __syncthreads();
  const uint32_t R = nR;
  if (tid == 0) {
    // lowest score level that still belongs to the first C
    uint32_t cum = 0;
    int thr = 0;
    if (R > (uint32_t)C) {
      for (int s = c.H; s >= 0; --s) {
        if (cum + hist[s] >= (uint32_t)C) {
          thr = s;
          break;
        }
        cum += hist[s];
      }
      need = (uint32_t)C - cum;  // members to take from level thr
    } else {
      thr = -1;  // everything
      need = 0;
    }
    s_thr = thr;
  }
  __syncthreads();
  const int thr = s_thr;
  const uint32_t tieN = thr >= 0 ? hist[thr] : 0;
  const bool ties_fit = tieN <= (uint32_t)kTieCap;
  // keep members above the level, collect the level's ids if they fit
  for_members(c, qk, qh, glo, gpre, e0, e1, sc, false, [&](uint32_t X, int score) {
    if (score > thr) {
      const uint32_t slot = atomicAdd(&nsel, 1u);
      sel[slot] = ((uint64_t)(c.H - score) << 32) | X;
    } else if (score == thr && ties_fit) {
      ties[atomicAdd(&ntie, 1u)] = X;
    }
  }, [&](int score) { return score > thr || (score == thr && ties_fit); });
  __syncthreads();
  if (thr >= 0) {
    if (ties_fit) {
      const int n2 = pow2_at_least((int)tieN);
      for (int i = tid + (int)tieN; i < n2; i += kPrThreads) ties[i] = 0xFFFFFFFFu;
      __syncthreads();
      bitonic_sort(ties, n2);
      const uint32_t base = nsel;
      for (uint32_t i = tid; i < need; i += kPrThreads)
        sel[base + i] = ((uint64_t)(c.H - thr) << 32) | ties[i];
      __syncthreads();
      if (tid == 0) nsel = base + need;
      __syncthreads();
    } else {
      // radix select of the need-th smallest id of level thr, one byte per pass
      if (tid == 0) prefix = 0;
      __syncthreads();
      for (int pass = 0; pass < 4; ++pass) {
        const int sh = 24 - 8 * pass;
        for (int i = tid; i < 256; i += kPrThreads) bhist[i] = 0;
        __syncthreads();
        const uint32_t pfx = prefix;
        for_members(c, qk, qh, glo, gpre, e0, e1, sc, false, [&](uint32_t X, int score) {
          if (score == thr && (pass == 0 || (X >> (sh + 8)) == (pfx >> (sh + 8))))
            atomicAdd(&bhist[(X >> sh) & 255], 1u);
        }, [&](int score) { return score == thr; });
        __syncthreads();
        if (tid == 0) {
          uint32_t cum = 0, nd = need;
          int byte = 0;
          for (; byte < 256; ++byte) {
            if (cum + bhist[byte] >= nd) break;
            cum += bhist[byte];
          }
          need = nd - cum;
          prefix = pfx | ((uint32_t)byte << sh);
        }
        __syncthreads();
      }
      const uint32_t T = prefix;  // the need-th smallest id of the level
      for_members(c, qk, qh, glo, gpre, e0, e1, sc, false, [&](uint32_t X, int score) {
        if (score == thr && X <= T) sel[atomicAdd(&nsel, 1u)] = ((uint64_t)(c.H - thr) << 32) | X;
      }, [&](int score) { return score == thr; });
      __syncthreads();
    }
  }
  const int ns = (int)nsel;
  for (int i = tid; i < ns; i += kPrThreads) out[i] = sel[i];
  if (tid == 0) {
    ws.nkeys[(int64_t)q * F + part] = (uint32_t)ns;
    ws.rpart[(int64_t)q * F + part] = R;
  }
}

// ---------------------------------------------------------------------------
// 3. merge
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPrThreads) void probe_merge_kernel(int C, int F, ProbeWs ws,
                                                                 int64_t* __restrict__ cand,
                                                                 int32_t* __restrict__ ncand,
                                                                 int64_t* __restrict__ r_size) {
  __shared__ uint64_t keys[kMergeCap];
  __shared__ uint32_t base[kMaxParts + 1];
  __shared__ int64_t rsum;
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid == 0) {
    uint32_t b = 0;
    int64_t r = 0;
    for (int f = 0; f < F; ++f) {
      base[f] = b;
      b += ws.nkeys[(int64_t)q * F + f];
      r += ws.rpart[(int64_t)q * F + f];
    }
    base[F] = b;
    rsum = r;
  }
  __syncthreads();
  const int total = (int)base[F];  // <= F C <= kMergeCap
  for (int f = 0; f < F; ++f) {
    const uint64_t* src = ws.keys + ((int64_t)q * F + f) * C;
    const int nf = (int)(base[f + 1] - base[f]);
    for (int i = tid; i < nf; i += kPrThreads) keys[base[f] + i] = src[i];
  }
  const int n2 = pow2_at_least(total > 0 ? total : 1);
  for (int i = tid + total; i < n2; i += kPrThreads) keys[i] = ~0ull;
  __syncthreads();
  bitonic_sort(keys, n2);
  const int ns = total < C ? total : C;
  int64_t* crow = cand + (int64_t)q * C;
  for (int i = tid; i < C; i += kPrThreads) crow[i] = i < ns ? (int64_t)(uint32_t)keys[i] : -1;
  if (tid == 0) {
    ncand[q] = ns;
    r_size[q] = rsum;
  }
}

size_t probe_workspace_bytes(int nq, int L, int C) { return probe_ws_bytes(nq, L, C); }

ssh_status probe_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int L,
                        const uint64_t* db_keys, const uint64_t* db_hv, int H,
                        const uint64_t* q_keys, const uint64_t* q_hv, int nq, int C, int64_t* cand,
                        int32_t* ncand, int64_t* r_size, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (L > kMaxL) return fail(SSH_EUNSUPPORTED, "ssh_probe: more than 64 tables");
  if (H > kMaxH) return fail(SSH_EUNSUPPORTED, "ssh_probe: more than 1024 hashes");
  if (nq == 0) return SSH_OK;
  if ((int64_t)nq * probe_parts(C) > (int64_t)INT32_MAX)
    return fail(SSH_EUNSUPPORTED, "ssh_probe: too many queries for one launch");
  if (ws_bytes < probe_ws_bytes(nq, L, C))
    return fail(SSH_EINVAL, "ssh_probe: workspace smaller than ssh_probe_workspace_bytes");
  ProbeCtx c{tab_keys, tab_ids, N, L, db_keys, db_hv, H};
  const ProbeWs w = probe_ws(ws, nq, L, C);
  const int F = probe_parts(C);
  probe_runs_kernel<<<nq, kWave, 0, stream>>>(c, q_keys, w);
  const size_t dyn = ((size_t)H + (H + 2) / 2 + (size_t)C) * 8;
  probe_part_kernel<<<(unsigned)((int64_t)nq * F), kPrThreads, dyn, stream>>>(c, q_keys, q_hv, C, F,
                                                                               w);
  probe_merge_kernel<<<nq, kPrThreads, 0, stream>>>(C, F, w, cand, ncand, r_size);
  return check_launch("ssh_probe");
}

}  // namespace ssh
