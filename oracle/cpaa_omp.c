/* FP64 CPU reference of CPAA and of the power method, plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: the multi-core CPU baseline of the benchmark, pinned
 * against the numpy oracle by tests/test_oracle_omp.py.  It shares nothing with
 * the HIP library (its own SpMV, coefficients and loops).
 *
 * P = A D^{-1} of an undirected graph (Sec. 2.1): (P y)_u = sum_{v in N(u)} y_v / d_v,
 * the division of Alg. 1's inner loop.
 *
 * cpaa_ref_cpaa: x_M = (c_0/2) b + sum_{k=1..M} c_k T_k(P) b (eq. 3.1 applied to b),
 *   rounds as in Alg. 1: round 1 forms T' = P T; round k >= 2 forms T'' = 2 P T' - T,
 *   adds c_k T'' to the sum and rotates T <- T', T' <- T''.  Coefficients from
 *   Prop. 1: c_0 = 2 / sqrt(1 - c^2), c_k = c_0 beta^k, beta = (1 - sqrt(1 - c^2)) / c.
 * cpaa_ref_power: x_0 = (1-c) p, x_{t+1} = c P x_t + (1-c) p (the fixed point of
 *   eq. 2.1 for an undirected graph), stopped once c ||x_{t+1} - x_t||_1 / (1-c) <= tol
 *   (a bound on the error of x_{t+1}, since ||(I - cP)^{-1}||_1 = 1/(1-c)) or after
 *   max_iter steps; returns the steps taken.
 *
 * Both take the CSR pattern (int32, rows sorted or not), run on `threads` OpenMP
 * threads (<= 0: the OpenMP default) and write x[n].  Return -1 on a bad argument or
 * allocation failure.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* out = P y: w_v = y_v / d_v once per vertex (the same quotient Alg. 1 forms per
 * entry), then out_u = sum_{v in N(u)} w_v.  w is caller scratch [n]. */
static void apply_p(int n, const int32_t* rp, const int32_t* ci, const double* deg,
                    const double* y, double* w, double* out) {
#pragma omp parallel for schedule(static)
  for (int v = 0; v < n; ++v) w[v] = y[v] / deg[v];
#pragma omp parallel for schedule(dynamic, 4096)
  for (int u = 0; u < n; ++u) {
    double s = 0.0;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) s += w[ci[j]];
    out[u] = s;
  }
}

static double* degrees(int n, const int32_t* rp) {
  double* d = (double*)malloc((size_t)n * sizeof(double));
  if (!d) return NULL;
#pragma omp parallel for schedule(static)
  for (int u = 0; u < n; ++u) d[u] = (double)(rp[u + 1] - rp[u]);
  return d;
}

int cpaa_ref_cpaa(int n, const int32_t* rp, const int32_t* ci, double c, const double* b, int M,
                  double* x, int threads) {
  if (n <= 0 || !rp || !ci || !b || !x || M < 0 || !(c > 0.0 && c < 1.0)) return -1;
  if (threads > 0) omp_set_num_threads(threads);
  const double s = sqrt(1.0 - c * c);
  const double beta = (1.0 - s) / c;
  const double c0 = 2.0 / s;
  double* deg = degrees(n, rp);
  double* w = (double*)malloc((size_t)n * sizeof(double));
  double* t_prev = (double*)malloc((size_t)n * sizeof(double));
  double* t_cur = (double*)malloc((size_t)n * sizeof(double));
  double* t_next = (double*)malloc((size_t)n * sizeof(double));
  if (!deg || !w || !t_prev || !t_cur || !t_next) {
    free(deg);
    free(w);
    free(t_prev);
    free(t_cur);
    free(t_next);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int u = 0; u < n; ++u) {
    t_prev[u] = b[u];
    x[u] = (c0 / 2.0) * b[u];
  }
  if (M >= 1) {
    apply_p(n, rp, ci, deg, t_prev, w, t_cur);           /* round 1: T_1 b = P b */
    const double c1 = c0 * beta;
#pragma omp parallel for schedule(static)
    for (int u = 0; u < n; ++u) x[u] += c1 * t_cur[u];
  }
  double ck = c0 * beta;
  for (int k = 2; k <= M; ++k) {
    ck *= beta;
    apply_p(n, rp, ci, deg, t_cur, w, t_next);
#pragma omp parallel for schedule(static)
    for (int u = 0; u < n; ++u) {
      t_next[u] = 2.0 * t_next[u] - t_prev[u];      /* T'' = 2 P T' - T */
      x[u] += ck * t_next[u];
    }
    double* r = t_prev;                               /* T <- T', T' <- T'' */
    t_prev = t_cur;
    t_cur = t_next;
    t_next = r;
  }
  free(deg);
  free(w);
  free(t_prev);
  free(t_cur);
  free(t_next);
  return 0;
}

int cpaa_ref_power(int n, const int32_t* rp, const int32_t* ci, double c, const double* p,
                   double tol, int max_iter, double* x, int threads) {
  if (n <= 0 || !rp || !ci || !p || !x || max_iter < 0 || !(c > 0.0 && c < 1.0)) return -1;
  if (threads > 0) omp_set_num_threads(threads);
  double* deg = degrees(n, rp);
  double* w = (double*)malloc((size_t)n * sizeof(double));
  double* px = (double*)malloc((size_t)n * sizeof(double));
  if (!deg || !w || !px) {
    free(deg);
    free(w);
    free(px);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int u = 0; u < n; ++u) x[u] = (1.0 - c) * p[u];
  int it = 0;
  while (it < max_iter) {
    apply_p(n, rp, ci, deg, x, w, px);
    double diff = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : diff)
    for (int u = 0; u < n; ++u) {
      const double xn = c * px[u] + (1.0 - c) * p[u];
      diff += fabs(xn - x[u]);
      x[u] = xn;
    }
    ++it;
    if (c * diff / (1.0 - c) <= tol) break;
  }
  free(deg);
  free(w);
  free(px);
  return it;
}
