/* Banded dynamic time warping in float64 -- CPU oracle, test infrastructure only.
 *
 * Follows Section 2.1 of Luo & Shrivastava (DTW): the cost of aligning q_i
 * with x_j is the squared difference, a warping path moves by (1,0), (0,1)
 * or (1,1) from (0,0) to (lq-1, lx-1), and the distance is the square root
 * of the smallest total cost.  A Sakoe-Chiba band |i - j| <= r restricts the
 * path; no path exists when |lq - lx| > r and the distance is +inf.
 *
 * The dynamic program is the textbook one, row by row:
 *   D(0,0) = cost(0,0)
 *   D(i,j) = cost(i,j) + min(D(i-1,j), D(i,j-1), D(i-1,j-1))
 * with cells outside the matrix or the band at +inf.  Built with
 * -ffp-contract=off, so cost(i,j) = d*d and the sum are separately rounded.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>

static double min3(double a, double b, double c) {
  double m = a < b ? a : b;
  return m < c ? m : c;
}

double oracle_dtw(const float* q, int64_t lq, const float* x, int64_t lx, int64_t r) {
  if (lq <= 0 || lx <= 0) return INFINITY;
  if (llabs(lq - lx) > r) return INFINITY;
  double* prev = (double*)malloc((size_t)lx * sizeof(double));
  double* cur = (double*)malloc((size_t)lx * sizeof(double));
  for (int64_t j = 0; j < lx; j++) prev[j] = INFINITY;
  for (int64_t i = 0; i < lq; i++) {
    for (int64_t j = 0; j < lx; j++) cur[j] = INFINITY;
    int64_t lo = i - r > 0 ? i - r : 0;
    int64_t hi = i + r < lx - 1 ? i + r : lx - 1;
    for (int64_t j = lo; j <= hi; j++) {
      double d = (double)q[i] - (double)x[j];
      double cost = d * d;
      double best;
      if (i == 0 && j == 0) {
        best = 0.0;
      } else {
        double up = i > 0 ? prev[j] : INFINITY;
        double left = j > 0 ? cur[j - 1] : INFINITY;
        double diag = (i > 0 && j > 0) ? prev[j - 1] : INFINITY;
        best = min3(up, left, diag);
      }
      cur[j] = cost + best;
    }
    double* t = prev;
    prev = cur;
    cur = t;
  }
  double total = prev[lx - 1];
  free(prev);
  free(cur);
  return sqrt(total);
}

/* Distances of every (query, candidate) pair; cand is [nq][C], ncand[i]
 * entries valid per row; dist[i*C + c] is written for c < ncand[i].
 * The radius of a pair is floor(band_frac * max(lq, lx)) in double. */
void oracle_dtw_pairs(const float* q, const int64_t* q_off, int64_t nq, const float* db,
                      const int64_t* db_off, const int64_t* cand, const int32_t* ncand,
                      int64_t C, float band_frac, double* dist) {
  int64_t total = nq * C;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t p = 0; p < total; p++) {
    int64_t i = p / C, c = p % C;
    if (c >= ncand[i]) continue;
    int64_t id = cand[p];
    int64_t lq = q_off[i + 1] - q_off[i];
    int64_t lx = db_off[id + 1] - db_off[id];
    int64_t mx = lq > lx ? lq : lx;
    int64_t r = (int64_t)floor((double)band_frac * (double)mx);
    dist[p] = oracle_dtw(q + q_off[i], lq, db + db_off[id], lx, r);
  }
}

/* Number of threads the parallel loop above runs on. */
int32_t oracle_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
