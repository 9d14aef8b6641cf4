// Host build of the library's Matern evaluation (matern.hpp: closed forms for
// nu = 1/2, 3/2, 5/2; otherwise x^mu K_mu by the trapezoidal rule on the
// integral representation and the upward recurrence; Section 1, eq. (2)),
// with the parameter setup of common.hpp, run by tests/test_host_matern.py.
// The device build uses the same code with the device's exp and log.
//
// Reads lines "sigma2 ell nu h" from stdin and prints, for each, the
// covariance in float64 and in float32 (the mixed-precision path).
#include <cstdio>

#include "../../paper_2104_07146_amd/csrc/matern.hpp"

int main() {
  double s2, ell, nu, h;
  while (std::scanf("%lf %lf %lf %lf", &s2, &ell, &nu, &h) == 4) {
    const hmle::MaternParams mp = hmle::matern_params(hmle_theta{s2, ell, nu, 0.0});
    const double v64 = hmle::matern_value<double>(h, mp);
    const float v32 = hmle::matern_value<float>((float)h, mp);
    std::printf("%.17g %.9g\n", v64, (double)v32);
  }
  return 0;
}
