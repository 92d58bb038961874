// Weighted MinHash of the shingle sets by consistent weighted sampling
// (Section 4.3, and Section 2, eqs. WJaccardDef / CollProb), following Ioffe's
// improved consistent weighted sampling, the sampler the paper cites.
//
// For hash j and token k of weight S (draws r ~ Gamma(2,1), ln c, beta ~ U[0,1)):
//     t    = floor(ln S / r + beta)
//     ln y = r (t - beta)
//     ln a = ln c - ln y - r
// k* = argmin_k ln a (ties to the smaller k), hv = min(t*, 2^48-1) << 16 | k*.
// Every step is one correctly rounded float64 operation, in this order; the
// library is compiled without floating-point contraction so no step fuses.
// ln S comes from a table of correctly rounded logarithms prepared once on
// the device by a double-double evaluation (and is evaluated the same way on
// the fly for the rare count beyond the table).  A token of weight 1 has
// ln S = 0, t = 0 and ln a = (ln c - r * (0 - beta)) - r, which the prepare
// kernel stores per (k, j) so the common case is one 8-byte load.
#include <cmath>

#include "common.hpp"

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

// ---------------------------------------------------------------------------
// prepare: lnS table and the weight-1 ln a of every (k, j)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cws_prepare_kernel(const double* __restrict__ r,
                                                          const double* __restrict__ lnc,
                                                          const double* __restrict__ beta,
                                                          int64_t cells, double* __restrict__ a1,
                                                          double* __restrict__ lnS, int* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
    const double rr = r[i], bb = beta[i], lc = lnc[i];
    if (!(rr > 0.0) || !(rr < INFINITY) || !(bb >= 0.0) || !(bb < 1.0) || !(__builtin_fabs(lc) < INFINITY))
      atomicOr(err, 2);
    const double t = 0.0;  // floor(0 / r + beta) for beta in [0, 1)
    const double ln_y = rr * (t - bb);
    a1[i] = (lc - ln_y) - rr;
  }
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < SSH_LNS_ENTRIES; s += stride)
    lnS[s] = s == 0 ? -INFINITY : ln_integer((double)s);
}

// ---------------------------------------------------------------------------
// main: one thread per (series, hash)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cws_kernel(
    const uint32_t* __restrict__ codes, const uint32_t* __restrict__ counts,
    const int64_t* __restrict__ hist_off, const int32_t* __restrict__ n_distinct, int64_t N, int H,
    const double* __restrict__ r, const double* __restrict__ lnc, const double* __restrict__ beta,
    const double* __restrict__ a1, const double* __restrict__ lnS, uint64_t* __restrict__ hv) {
  const int64_t total = N * (int64_t)H;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int64_t s = g / H;
    const int j = (int)(g - s * H);
    const int D = n_distinct[s];
    if (D <= 0) {
      hv[g] = SSH_HV_EMPTY;
      continue;
    }
    const int64_t ho = hist_off[s];
    double best = INFINITY, bt = 0.0;
    uint32_t bk = 0;
    for (int d = 0; d < D; ++d) {
      const uint32_t k = codes[ho + d];
      const uint32_t c = counts[ho + d];
      const int64_t idx = (int64_t)k * H + j;
      double la, t;
      if (c == 1) {
        la = a1[idx];
        t = 0.0;
      } else {
        const double ls = c < (uint32_t)SSH_LNS_ENTRIES ? lnS[c] : ln_integer((double)c);
        const double rr = r[idx], bb = beta[idx];
        t = __builtin_floor(ls / rr + bb);
        const double ln_y = rr * (t - bb);
        la = (lnc[idx] - ln_y) - rr;
      }
      if (la < best) {
        best = la;
        bk = k;
        bt = t;
      }
    }
    const double tmax = 281474976710655.0;  // 2^48 - 1
    const uint64_t tt = (uint64_t)(bt < tmax ? bt : tmax);
    hv[g] = (tt << 16) | (uint64_t)bk;
  }
}

__device__ int g_cws_err;

int take_cws_err() {
  int v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_cws_err), sizeof(int)) != hipSuccess) return -1;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_cws_err), &z, sizeof(int)) != hipSuccess) return -1;
  return v;
}

ssh_status cws_prepare_launch(const ssh_cws_tables* tab, hipStream_t stream) {
  int* err = nullptr;
  if (hipGetSymbolAddress((void**)&err, HIP_SYMBOL(g_cws_err)) != hipSuccess)
    return fail(SSH_EDEVICE, "ssh_cws_prepare: cannot resolve error flag");
  const int64_t cells = ((int64_t)1 << tab->n) * tab->H;
  cws_prepare_kernel<<<grid_for(cells, 256, 4096), 256, 0, stream>>>(tab->r, tab->lnc, tab->beta,
                                                                      cells, tab->a1, tab->lnS, err);
  return check_launch("ssh_cws_prepare");
}

ssh_status cws_launch(const uint32_t* codes, const uint32_t* counts, const int64_t* hist_off,
                      const int32_t* n_distinct, int64_t N, const ssh_cws_tables* tab, uint64_t* hv,
                      hipStream_t stream) {
  if (N == 0) return SSH_OK;
  const int64_t total = N * (int64_t)tab->H;
  cws_kernel<<<grid_for(total, 256, 1 << 20), 256, 0, stream>>>(
      codes, counts, hist_off, n_distinct, N, tab->H, tab->r, tab->lnc, tab->beta, tab->a1,
      tab->lnS, hv);
  return check_launch("ssh_cws");
}

}  // namespace ssh
