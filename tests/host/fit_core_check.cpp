// Host-only driver of the optimiser in fit.cpp (Section 2, "Maximization of
// the log-likelihood"; Section 5.1 coordinates), built with g++ by
// tests/test_host_fit.py. The evaluation entry points that fit.cpp calls are
// replaced here by a test double whose "log-likelihood" is a smooth analytic
// function of log(theta), so the search runs without a GPU and every point it
// evaluates can be compared with an independent Nelder-Mead (SciPy's) started
// from the same simplex. Nothing here is the method's arithmetic.
//
// Usage: fit_core_check PROFILE SIGMA2 ELL NU TAU2 STEP TOL MAX_ITER TAU2_FLOOR ELL_BAND
//   PROFILE     0: four-parameter fit, 1: variance profiled out
//   SIGMA2..    start point; SIGMA2 = 0 means the default start
//   TAU2_FLOOR  the factorisation reports "not positive definite" when the
//               nugget tau2 is below it (exercises the start back-off)
//   ELL_BAND    when > 0, the factorisation also fails for ell in
//               [ELL_BAND, 1.15 ELL_BAND): a contraction landing in the band
//               fails, so the search shrinks
//   COUNT       optional (after STOP_AT, which must then be 0): when > 0, the
//               fit also runs through hmle_fit_batch with COUNT candidates per
//               batched evaluation ("batch status s2 ell nu tau2 evals iters
//               failed converged logL rounds")
//   STOP_AT     optional: when > 0, the fit runs through hmle_fit_resumable,
//               first stopped after STOP_AT iterations ("stopped status evals
//               iters"), then continued from its checkpoint; a further call
//               with the final checkpoint prints "again ..." like "result",
//               and the checkpoint offered to the other kind of search prints
//               "mismatch status", and the same search on other data
//               "otherdata status"
// Output: one line "eval s2 ell nu tau2" per evaluation the double served, then
// "result status s2 ell nu tau2 evals iters failed converged logL".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/hmle.h"
#include "../../paper_2104_07146_amd/csrc/fit_support.hpp"

namespace {

const double kN = 1000.0;
int32_t g_count = 0;
double g_floor = 0.0;
double g_band = 0.0;
hmle_theta g_theta{};

double centre(int i) {
  static const double c[4] = {std::log(1.3), std::log(0.12), std::log(0.7), std::log(0.02)};
  return c[i];
}

// four-parameter objective: logL = -(1/2 u^T A u + u0^4 / 20), u = log(theta) - centre
double full_loglik(const hmle_theta& t) {
  static const double A[4][4] = {{4, 1, 0.5, 0}, {1, 3, 0.8, 0.2}, {0.5, 0.8, 2, 0.1}, {0, 0.2, 0.1, 1}};
  const double u[4] = {std::log(t.sigma2) - centre(0), std::log(t.range) - centre(1), std::log(t.nu) - centre(2),
                       std::log(t.tau2) - centre(3)};
  double q = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) q += u[i] * A[i][j] * u[j];
  return -(0.5 * q + u[0] * u[0] * u[0] * u[0] / 20.0);
}

// profiled objective (called at sigma2 = 1, tau2 = r): log-determinant h1 and
// quadratic form n exp(h2), v = log(ell, nu, r) - centre
void profile_parts(const hmle_theta& t, double* h1, double* h2) {
  static const double B[3][3] = {{2, 0.3, 0.1}, {0.3, 1, 0.2}, {0.1, 0.2, 0.5}};
  const double v[3] = {std::log(t.range) - centre(1), std::log(t.nu) - centre(2), std::log(t.tau2) - centre(3)};
  double q = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) q += v[i] * B[i][j] * v[j];
  *h1 = 10.0 + 50.0 * q;
  *h2 = 0.1 * (v[0] * v[0] + v[0] * v[2] + 0.5 * v[2] * v[2]) + 0.05 * v[1] * v[1] + 0.01 * v[0];
}

}  // namespace

extern "C" {

void hmle_default_fit_opts(hmle_fit_opts* o) {
  o->max_iter = 400;
  o->tol = 1e-4;
  o->step = 1.0;
  o->use_backoff = 1;
  o->report_every = 0;
  o->profile_variance = 0;
}

hmle_status hmle_sizes(hmle_problem, int64_t sizes[6]) {
  sizes[0] = (int64_t)kN;
  for (int i = 1; i < 6; ++i) sizes[i] = 0;
  return HMLE_OK;
}

hmle_status hmle_assemble(hmle_problem, const hmle_theta* theta) {
  g_theta = *theta;
  return HMLE_OK;
}

hmle_status hmle_factor(hmle_problem) {
  const bool band = g_band > 0 && g_theta.range >= g_band && g_theta.range < 1.15 * g_band;
  return g_theta.tau2 < g_floor || band ? HMLE_E_NOT_SPD : HMLE_OK;
}

hmle_status hmle_loglik(hmle_problem, const double*, double out[3]) {
  const hmle_theta& t = g_theta;
  std::printf("eval %.17g %.17g %.17g %.17g\n", t.sigma2, t.range, t.nu, t.tau2);
  double h1, h2;
  profile_parts(t, &h1, &h2);
  out[0] = full_loglik(t);
  out[1] = h1;
  out[2] = kN * std::exp(h2);
  return HMLE_OK;
}

// The batched evaluation of g_count points: each as hmle_assemble +
// hmle_factor + hmle_loglik would give it, its status per point.
hmle_status hmle_eval_batch(hmle_problem p, const hmle_theta* thetas, const double* z, double* out, hmle_status* st) {
  for (int32_t i = 0; i < g_count; ++i) {
    hmle_assemble(p, &thetas[i]);
    st[i] = hmle_factor(p);
    if (st[i] == HMLE_OK) {
      const hmle_theta& t = thetas[i];
      double h1, h2;
      profile_parts(t, &h1, &h2);
      out[3 * i] = full_loglik(t);
      out[3 * i + 1] = h1;
      out[3 * i + 2] = kN * std::exp(h2);
    } else {
      out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = NAN;
    }
  }
  (void)z;
  return HMLE_OK;
}

}  // extern "C"

namespace hmle {
hmle_status candidate_layout(hmle_problem, int32_t* count, int64_t* n1) {
  if (g_count < 1) return HMLE_E_INVALID;
  *count = g_count;
  *n1 = (int64_t)kN;
  return HMLE_OK;
}
// fit.cpp's batched fit keeps one copy of z per candidate in the batch's
// device memory; here that memory is host memory
hmle_status candidate_data(hmle_problem, const double* z, int32_t count, int64_t n1, double** out) {
  static std::vector<double> zz;
  zz.resize((size_t)count * n1);
  for (int32_t k = 0; k < count; ++k) std::memmove(zz.data() + (size_t)k * n1, z, n1 * sizeof(double));
  *out = zz.data();
  return HMLE_OK;
}
// the data's fingerprint (here z is host memory of kN values)
hmle_status fit_fingerprint(hmle_problem, const double* z, uint32_t* out) {
  uint32_t x = 2166136261u;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(z);
  for (size_t i = 0; i < (size_t)kN * sizeof(double); ++i) x = (x ^ b[i]) * 16777619u;
  *out = x;
  return HMLE_OK;
}
}  // namespace hmle

int main(int argc, char** argv) {
  if (argc < 11 || argc > 13) {
    std::fprintf(stderr, "usage: %s PROFILE SIGMA2 ELL NU TAU2 STEP TOL MAX_ITER TAU2_FLOOR ELL_BAND [STOP_AT [COUNT]]\n",
                 argv[0]);
    return 2;
  }
  hmle_fit_opts o;
  hmle_default_fit_opts(&o);
  o.profile_variance = std::atoi(argv[1]);
  const hmle_theta start{std::atof(argv[2]), std::atof(argv[3]), std::atof(argv[4]), std::atof(argv[5])};
  o.step = std::atof(argv[6]);
  o.tol = std::atof(argv[7]);
  o.max_iter = std::atoi(argv[8]);
  g_floor = std::atof(argv[9]);
  g_band = std::atof(argv[10]);
  const int stop_at = argc >= 12 ? std::atoi(argv[11]) : 0;
  g_count = argc == 13 ? std::atoi(argv[12]) : 0;
  std::vector<double> zbuf((size_t)kN, 0.0);
  int dummy = 0;
  hmle_problem p = reinterpret_cast<hmle_problem>(&dummy);
  const double* z = zbuf.data();
  const hmle_theta* st = start.sigma2 > 0 ? &start : nullptr;
  hmle_theta th{};
  hmle_fit_report rep{};
  auto print = [&](const char* what, hmle_status s) {
    std::printf("%s %d %.17g %.17g %.17g %.17g %d %d %d %d %.17g\n", what, (int)s, th.sigma2, th.range, th.nu,
                th.tau2, rep.evals, rep.iters, rep.failed_evals, rep.converged, rep.logL);
  };
  if (stop_at <= 0) {
    print("result", hmle_fit(p, z, st, &o, &th, &rep));
    if (g_count > 0) {
      int32_t rounds = 0;
      const hmle_status sb = hmle_fit_batch(p, z, st, &o, &th, &rep, &rounds);
      std::printf("batch %d %.17g %.17g %.17g %.17g %d %d %d %d %.17g %d\n", (int)sb, th.sigma2, th.range, th.nu,
                  th.tau2, rep.evals, rep.iters, rep.failed_evals, rep.converged, rep.logL, rounds);
    }
    return 0;
  }
  std::vector<unsigned char> state(HMLE_FIT_STATE_BYTES, 0);
  hmle_fit_opts first = o;
  first.max_iter = stop_at;
  const hmle_status s1 = hmle_fit_resumable(p, z, st, &first, state.data(), (int64_t)state.size(), &th, &rep);
  std::printf("stopped %d %d %d\n", (int)s1, rep.evals, rep.iters);
  print("result", hmle_fit_resumable(p, z, st, &o, state.data(), (int64_t)state.size(), &th, &rep));
  std::fflush(stdout);
  print("again", hmle_fit_resumable(p, z, st, &o, state.data(), (int64_t)state.size(), &th, &rep));
  hmle_fit_opts other = o;
  other.profile_variance = !o.profile_variance;
  std::printf("mismatch %d\n", (int)hmle_fit_resumable(p, z, st, &other, state.data(), (int64_t)state.size(), &th,
                                                        &rep));
  // the same search on other data (one value changed) refuses the checkpoint
  std::vector<double> z2(zbuf);
  z2[(size_t)kN / 2] = 1.0;
  std::printf("otherdata %d\n", (int)hmle_fit_resumable(p, z2.data(), st, &o, state.data(), (int64_t)state.size(), &th,
                                                         &rep));
  return 0;
}
