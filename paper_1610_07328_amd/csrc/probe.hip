// Query probe (Algorithm 2: the retrieved set R is the union, over the hash
// tables, of the query's bucket in each), then ranking of R.
//
// One workgroup per query.
//  1. Per table, two binary searches find the run of entries whose high key
//     half equals the query's; entries of the run with the full key are the
//     bucket.
//  2. A member X of R is counted once, at the first table whose key matches
//     (X's keys in earlier tables are compared with the query's), so no
//     de-duplication structure is needed.  Its score is the number of hash
//     values it shares with the query.
//  3. Members are ordered by (score desc, id asc) through the composite key
//     (H - score) << 32 | id.  A histogram of scores finds the score level
//     holding the C-th member; members above it are kept, and among that
//     level the smallest ids are taken (sorted in LDS when they fit, else by a
//     radix select over id bytes).  The C kept keys are bitonic-sorted in LDS.
#include "common.hpp"

namespace ssh {

constexpr int kPrThreads = 256;
constexpr int kMaxL = 64;
constexpr int kMaxH = 1024;
constexpr int kTieCap = 4096;

struct ProbeCtx {
  const uint64_t* tab_keys;
  const uint32_t* tab_ids;
  int64_t N;
  int L;
  const uint64_t* db_keys;
  const uint64_t* db_hv;
  int H;
};

// Number of the H hash values of X equal to the query's (qh in LDS): the
// row is read 16 bytes at a time, eight loads in flight.
__device__ __forceinline__ int member_score(const ProbeCtx& c, uint32_t X, const uint64_t* qh) {
  const uint64_t* xh = c.db_hv + (int64_t)X * c.H;
  int score = 0;
  int j = 0;
  if ((c.H & 1) == 0 && ((uintptr_t)c.db_hv & 15) == 0) {  // rows are 16-byte aligned
    const ulonglong2* x2 = reinterpret_cast<const ulonglong2*>(xh);
    for (; j + 16 <= c.H; j += 16) {
      ulonglong2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = x2[j / 2 + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) score += (v[u].x == qh[j + 2 * u]) + (v[u].y == qh[j + 2 * u + 1]);
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
  if (c.tab_keys[idx] != qk[l]) return -1;
  const uint32_t X = c.tab_ids[idx];
  for (int l2 = 0; l2 < l; ++l2)
    if (c.db_keys[(int64_t)X * c.L + l2] == qk[l2]) return -1;
  return X;
}

constexpr int kScoreCap = 16384;          // entries whose scores are kept in LDS
constexpr uint16_t kNotMember = 0xFFFFu;

// Visit every member of R (once each) with its score.  With `sc` set, the
// first visit records every entry's score (kNotMember for non-members) and
// later visits read it instead of re-scoring.
template <typename F>
__device__ __forceinline__ void for_members(const ProbeCtx& c, const uint64_t* qk, const uint64_t* qh,
                                            const int64_t* glo, const int64_t* gpre, int64_t G,
                                            uint16_t* sc, bool first, F&& f) {
  for (int64_t e = threadIdx.x; e < G; e += kPrThreads) {
    if (sc && !first) {
      const uint16_t v = sc[e];
      if (v == kNotMember) continue;
      int l = 0;
      while (l + 1 < c.L && gpre[l + 1] <= e) ++l;
      const uint32_t X = c.tab_ids[(int64_t)l * c.N + glo[l] + (e - gpre[l])];
      f(X, (int)v);
      continue;
    }
    const int64_t X = entry_member(c, qk, glo, gpre, e);
    if (X < 0) {
      if (sc) sc[e] = kNotMember;
      continue;
    }
    const int score = member_score(c, (uint32_t)X, qh);
    if (sc) sc[e] = (uint16_t)score;
    f((uint32_t)X, score);
  }
}

__device__ void bitonic_sort_u64(uint64_t* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += kPrThreads) {
        const int p = i ^ j;
        if (p > i) {
          const uint64_t x = a[i], y = a[p];
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

__device__ void bitonic_sort_u32(uint32_t* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += kPrThreads) {
        const int p = i ^ j;
        if (p > i) {
          const uint32_t x = a[i], y = a[p];
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

__device__ __forceinline__ int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

__global__ __launch_bounds__(kPrThreads) void probe_kernel(ProbeCtx c, const uint64_t* __restrict__ q_keys,
                                                           const uint64_t* __restrict__ q_hv, int C,
                                                           int64_t* __restrict__ cand,
                                                           int32_t* __restrict__ ncand,
                                                           int64_t* __restrict__ r_size) {
  __shared__ uint64_t qk[kMaxL];
  __shared__ uint64_t qh[kMaxH];
  __shared__ int64_t glo[kMaxL];
  __shared__ int64_t gpre[kMaxL + 1];
  __shared__ uint32_t hist[kMaxH + 1];
  __shared__ uint32_t bhist[256];
  __shared__ uint64_t sel[SSH_MAX_C];
  __shared__ uint32_t ties[kTieCap];
  __shared__ uint16_t sc_buf[kScoreCap];
  __shared__ uint32_t nR, nsel, ntie;
  __shared__ int s_thr;
  __shared__ uint32_t prefix, need;

  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < c.L; i += kPrThreads) qk[i] = q_keys[(int64_t)q * c.L + i];
  for (int i = tid; i < c.H; i += kPrThreads) qh[i] = q_hv[(int64_t)q * c.H + i];
  for (int i = tid; i <= c.H; i += kPrThreads) hist[i] = 0;
  if (tid == 0) {
    nR = 0;
    nsel = 0;
    ntie = 0;
  }
  __syncthreads();
  int64_t* crow = cand + (int64_t)q * C;
  if (qk[0] == SSH_KEY_EMPTY || c.N == 0) {
    for (int i = tid; i < C; i += kPrThreads) crow[i] = -1;
    if (tid == 0) {
      ncand[q] = 0;
      r_size[q] = 0;
    }
    return;
  }
  // 1. run of equal high halves per table
  if (tid < c.L) {
    const int l = tid;
    const uint64_t* tk = c.tab_keys + (int64_t)l * c.N;
    const uint32_t hi = (uint32_t)(qk[l] >> 32);
    int64_t a = 0, b = c.N;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if ((uint32_t)(tk[mid] >> 32) < hi) a = mid + 1;
      else b = mid;
    }
    const int64_t lo = a;
    b = c.N;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if ((uint32_t)(tk[mid] >> 32) <= hi) a = mid + 1;
      else b = mid;
    }
    glo[l] = lo;
    gpre[l + 1] = a - lo;
  }
  __syncthreads();
  if (tid == 0) {
    gpre[0] = 0;
    for (int l = 0; l < c.L; ++l) gpre[l + 1] += gpre[l];
  }
  __syncthreads();
  const int64_t G = gpre[c.L];
  uint16_t* sc = G <= kScoreCap ? sc_buf : nullptr;
  // 2. score histogram over R
  for_members(c, qk, qh, glo, gpre, G, sc, true, [&](uint32_t X, int score) {
    (void)X;
    atomicAdd(&hist[score], 1u);
    atomicAdd(&nR, 1u);
  });
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
  // 3. keep members above the level, collect the level's ids if they fit
  __syncthreads();  // recorded scores visible to every thread
  for_members(c, qk, qh, glo, gpre, G, sc, false, [&](uint32_t X, int score) {
    if (score > thr) {
      const uint32_t slot = atomicAdd(&nsel, 1u);
      sel[slot] = ((uint64_t)(c.H - score) << 32) | X;
    } else if (score == thr && ties_fit) {
      ties[atomicAdd(&ntie, 1u)] = X;
    }
  });
  __syncthreads();
  if (thr >= 0) {
    if (ties_fit) {
      const int n2 = pow2_at_least((int)tieN);
      for (int i = tid + (int)tieN; i < n2; i += kPrThreads) ties[i] = 0xFFFFFFFFu;
      __syncthreads();
      bitonic_sort_u32(ties, n2);
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
        bhist[tid] = 0;
        __syncthreads();
        const uint32_t pfx = prefix;
        for_members(c, qk, qh, glo, gpre, G, sc, false, [&](uint32_t X, int score) {
          if (score == thr && (pass == 0 || (X >> (sh + 8)) == (pfx >> (sh + 8))))
            atomicAdd(&bhist[(X >> sh) & 255], 1u);
        });
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
      for_members(c, qk, qh, glo, gpre, G, sc, false, [&](uint32_t X, int score) {
        if (score == thr && X <= T) sel[atomicAdd(&nsel, 1u)] = ((uint64_t)(c.H - thr) << 32) | X;
      });
      __syncthreads();
    }
  }
  const int ns = (int)nsel;
  const int n2 = pow2_at_least(ns > 0 ? ns : 1);
  for (int i = tid + ns; i < n2; i += kPrThreads) sel[i] = ~0ull;
  __syncthreads();
  bitonic_sort_u64(sel, n2);
  for (int i = tid; i < C; i += kPrThreads) crow[i] = i < ns ? (int64_t)(uint32_t)sel[i] : -1;
  if (tid == 0) {
    ncand[q] = ns;
    r_size[q] = R;
  }
}

ssh_status probe_launch(const uint64_t* tab_keys, const uint32_t* tab_ids, int64_t N, int L,
                        const uint64_t* db_keys, const uint64_t* db_hv, int H,
                        const uint64_t* q_keys, const uint64_t* q_hv, int nq, int C, int64_t* cand,
                        int32_t* ncand, int64_t* r_size, hipStream_t stream) {
  if (L > kMaxL) return fail(SSH_EUNSUPPORTED, "ssh_probe: more than 64 tables");
  if (H > kMaxH) return fail(SSH_EUNSUPPORTED, "ssh_probe: more than 1024 hashes");
  if (nq == 0) return SSH_OK;
  ProbeCtx c{tab_keys, tab_ids, N, L, db_keys, db_hv, H};
  probe_kernel<<<nq, kPrThreads, 0, stream>>>(c, q_keys, q_hv, C, cand, ncand, r_size);
  return check_launch("ssh_probe");
}

}  // namespace ssh
