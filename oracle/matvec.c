/*
 * Exact covariance-vector product of the oracle -- TEST INFRASTRUCTURE ONLY.
 *
 *     y = C w,   C_ij = M(|s_i - s_j|) + tau^2 [i == j],
 *
 * with the Matern function of eq. (2) (Section 1) at the two smoothness values
 * where it has an elementary closed form (eq. (2) with h/ell and no sqrt(2 nu)):
 *     nu = 1/2:  M(h) = sigma^2 exp(-x),
 *     nu = 3/2:  M(h) = sigma^2 (1 + x) exp(-x),      x = h / ell,
 * and M(0) = sigma^2. Every entry is formed on the fly (O(n^2) work, O(n)
 * memory), so the product is exact up to rounding at sizes where C itself
 * does not fit in memory. Up to 16 vectors share each entry evaluation. Row i sums its terms in increasing j; rows are
 * independent and run in parallel (OpenMP). Distances by direct coordinate
 * differences. This file shares nothing with the GPU library.
 */
#include <math.h>

int oracle_cov_matvec(const double* pts, long n, int dim, double sigma2, double ell, int twice_nu, double tau2,
                      const double* w, long nrhs, double* y) {
  if (n < 0 || nrhs < 1 || nrhs > 16 || (dim != 2 && dim != 3) || !(ell > 0.0) || (twice_nu != 1 && twice_nu != 3))
    return 1;
  /* w and y: n x nrhs, row-major (the right-hand sides side by side) */
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    const double* pi = pts + i * dim;
    double acc[16];
    for (long r = 0; r < nrhs; ++r) acc[r] = 0.0;
    for (long j = 0; j < n; ++j) {
      const double* pj = pts + j * dim;
      double h2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        const double d = pi[k] - pj[k];
        h2 += d * d;
      }
      double m;
      if (h2 == 0.0) {
        m = sigma2;
      } else {
        const double x = sqrt(h2) / ell;
        m = twice_nu == 1 ? sigma2 * exp(-x) : sigma2 * (1.0 + x) * exp(-x);
      }
      for (long r = 0; r < nrhs; ++r) acc[r] += m * w[j * nrhs + r];
    }
    for (long r = 0; r < nrhs; ++r) y[i * nrhs + r] = acc[r] + tau2 * w[i * nrhs + r];
  }
  return 0;
}
