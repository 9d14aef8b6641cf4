// hmle_fit: maximum-likelihood estimation (Section 2, "Maximization of the
// log-likelihood"; Section 5.1 for the coordinates and the start point).
//
// The paper names a Brent-Dekker routine, which is one-dimensional. The four
// parameters are searched here with Nelder-Mead (reflection 1, expansion 2,
// contraction 1/2, shrink 1/2) on f = -L in the transformed coordinates
//   sigma = 2/1.1^s0, ell = 1/1.5^l0, nu = 1/1.2^n0, tau = 1/2^t0,
// initial simplex x0, x0 + step*e_i, stopped when every vertex lies within
// tol (max-norm) of the best one or after max_iter iterations. Each vertex is
// one assemble + factor + loglik on the GPU; a vertex outside the parameter
// box or whose matrix is not positive definite gets f = +inf.
//
// hmle_fit_batch runs the same iteration on a batch of copies of one point
// set: before each iteration the points it may need (reflection, the two
// contractions, expansion; the new vertices of a shrink; the initial simplex)
// are announced, and a missing value is computed together with up to
// count - 1 other announced points in one batched evaluation. Batched values
// equal single ones bit for bit, so the iterates, the estimate and the
// evaluation count are those of hmle_fit; only the number of GPU rounds drops.
//
// With opts.profile_variance the variance is profiled out: writing the nugget
// as tau^2 = r sigma^2, C = sigma^2 (R + r I) with R the unit-variance Matern
// correlation, and for fixed (ell, nu, r) eq. (1) is maximised by
// sigma^2 = q / n, q = Z^T (R + r I)^{-1} Z, which leaves
//   Lp(ell, nu, r) = -n/2 log(2 pi) - 1/2 log|R + r I| - n/2 log(q / n) - n/2.
// The iteration then runs over (ell0, nu0, tau0) only (tau = 1/2^tau0 now the
// ratio sqrt(r)), each vertex one factorisation of R + r I; the estimate is
// (q/n, ell, nu, r q/n) at the best vertex, which maximises eq. (1).
//
// hmle_fit_resumable keeps a checkpoint of the iteration in a caller-owned
// buffer: the sorted simplex, its values and the counters at the top of the
// loop where the fit stopped (max_iter or convergence). Called again with the
// buffer, it continues from there, so a fit stopped after k iterations and
// resumed evaluates exactly the points, and returns exactly the estimate and
// counts, of the same fit run without the stop.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hmle.h"
#include "fit_support.hpp"

namespace {

using Vec = std::array<double, 4>;

hmle_theta to_theta(const Vec& x) {
  const double sigma = 2.0 / std::pow(1.1, x[0]);
  const double ell = 1.0 / std::pow(1.5, x[1]);
  const double nu = 1.0 / std::pow(1.2, x[2]);
  const double tau = 1.0 / std::pow(2.0, x[3]);
  return hmle_theta{sigma * sigma, ell, nu, tau * tau};
}

Vec from_theta(const hmle_theta& t) {
  return Vec{std::log(2.0 / std::sqrt(t.sigma2)) / std::log(1.1), -std::log(t.range) / std::log(1.5),
             -std::log(t.nu) / std::log(1.2),
             t.tau2 > 0 ? -std::log(std::sqrt(t.tau2)) / std::log(2.0) : 60.0};
}

bool in_box(const hmle_theta& t) {
  return t.sigma2 >= 1e-6 && t.sigma2 <= 1e6 && t.range >= 1e-4 && t.range <= 10.0 && t.nu >= 0.05 && t.nu <= 8.0 &&
         t.tau2 >= 0.0 && t.tau2 <= 1e3;
}

// The objective of a vertex: -L (all four parameters) or -Lp (variance
// profiled out; the point is evaluated at sigma^2 = 1 and tau^2 = r).
struct Objective {
  bool profile = false;
  double n = 0.0;
  hmle_theta point(const Vec& x) const {
    hmle_theta t = to_theta(x);
    if (profile) t.sigma2 = 1.0;
    return t;
  }
  double value(const double out[3]) const {
    if (!profile) return -out[0];
    const double q = out[2];
    if (!(q > 0.0)) return INFINITY;
    return 0.5 * n * std::log(2.0 * M_PI) + 0.5 * out[1] + 0.5 * n * std::log(q / n) + 0.5 * n;
  }
};

// Counting and progress shared by both evaluators: every call of f counts as
// one evaluation, as in the sequential iteration.
struct Tally {
  Objective obj;
  int report_every = 0;
  int evals = 0, failed = 0;
  double best = INFINITY;
  hmle_theta best_th{};
  hmle_status hard = HMLE_OK;
  std::vector<std::pair<Vec, double>> quad;   // Z^T C^{-1} Z of every finite vertex (profiled fit)
  double quad_of(const Vec& x) const {
    for (const auto& e : quad)
      if (e.first == x) return e.second;
    return NAN;
  }
  void record(const Vec& x, double v) {
    if (v < best) { best = v; best_th = to_theta(x); }
    if (report_every > 0 && evals % report_every == 0)
      std::fprintf(stderr, "# hmle_fit: %d evaluations (%d failed), best logL %.10g at (%.6g, %.6g, %.6g, %.6g)\n",
                   evals, failed, -best, best_th.sigma2, best_th.range, best_th.nu, best_th.tau2);
  }
};

// One problem: each value is one assemble + factor + loglik.
struct SingleEval : Tally {
  hmle_problem p;
  const double* z;
  void expect(const Vec*, int) {}
  double operator()(const Vec& x) {
    const double v = value(x);
    record(x, v);
    return v;
  }
  double value(const Vec& x) {
    const hmle_theta th = obj.point(x);
    ++evals;
    if (!in_box(th) || !std::isfinite(th.sigma2) || !std::isfinite(th.tau2)) { ++failed; return INFINITY; }
    hmle_status s = hmle_assemble(p, &th);
    if (s == HMLE_OK) s = hmle_factor(p);
    double out[3];
    if (s == HMLE_OK) s = hmle_loglik(p, z, out);
    if (s == HMLE_E_NOT_SPD) { ++failed; return INFINITY; }
    if (s != HMLE_OK) {
      if (hard == HMLE_OK) hard = s;
      ++failed;
      return INFINITY;
    }
    const double v = obj.value(out);
    if (!std::isfinite(out[0]) || !std::isfinite(v)) { ++failed; return INFINITY; }
    quad.push_back({x, out[2]});
    return v;
  }
};

// A batch of `count` copies: announced points are evaluated lazily, up to
// `count` per batched evaluation (graph replay); zz holds z once per copy.
struct BatchEval : Tally {
  hmle_problem p;
  const double* zz;
  int count;
  int rounds = 0, computed = 0;
  std::vector<Vec> want;                 // announced points, in priority order
  std::vector<std::pair<Vec, double>> have;   // computed values of this iteration
  std::vector<hmle_theta> th;
  std::vector<double> out;
  std::vector<hmle_status> st;
  void expect(const Vec* xs, int k) {
    want.assign(xs, xs + k);
    have.clear();
  }
  const double* find(const Vec& x) const {
    for (const auto& h : have)
      if (h.first == x) return &h.second;
    return nullptr;
  }
  double operator()(const Vec& x) {
    ++evals;
    const hmle_theta t = obj.point(x);
    double v;
    if (!in_box(t) || !std::isfinite(t.sigma2) || !std::isfinite(t.tau2)) {
      v = INFINITY;
    } else {
      const double* c = find(x);
      if (!c) {
        compute(x);
        c = find(x);
      }
      v = c ? *c : INFINITY;
    }
    if (!std::isfinite(v)) ++failed;
    record(x, v);
    return v;
  }
  // x and up to count - 1 other announced, not yet computed, in-box points
  void compute(const Vec& x) {
    std::vector<Vec> pts{x};
    for (const Vec& w : want) {
      if ((int)pts.size() == count) break;
      if (w == x || find(w)) continue;
      bool dup = false;
      for (const Vec& q : pts) dup = dup || q == w;
      const hmle_theta t = obj.point(w);
      if (!dup && in_box(t) && std::isfinite(t.sigma2) && std::isfinite(t.tau2)) pts.push_back(w);
    }
    th.assign(count, obj.point(pts[0]));    // unused copies repeat the first point
    for (size_t i = 0; i < pts.size(); ++i) th[i] = obj.point(pts[i]);
    out.assign(3 * (size_t)count, 0.0);
    st.assign(count, HMLE_OK);
    ++rounds;
    computed += (int)pts.size();
    const hmle_status s = hmle_eval_batch(p, th.data(), zz, out.data(), st.data());
    if (s != HMLE_OK) {
      if (hard == HMLE_OK) hard = s;
      for (const Vec& q : pts) have.push_back({q, INFINITY});
      return;
    }
    for (size_t i = 0; i < pts.size(); ++i) {
      double v = INFINITY;
      if (st[i] == HMLE_OK && std::isfinite(out[3 * i])) {
        v = obj.value(&out[3 * i]);
        if (std::isfinite(v)) quad.push_back({pts[i], out[3 * i + 2]});
        else v = INFINITY;
      } else if (st[i] != HMLE_E_NOT_SPD && st[i] != HMLE_OK && hard == HMLE_OK) {
        hard = st[i];
      }
      have.push_back({pts[i], v});
    }
  }
};

// Checkpoint of the iteration at the top of its loop (simplex sorted by
// value): vertices, their objective values, their quadratic forms Z^T C^{-1} Z
// (used by the profiled fit's estimate), the counters and the best value.
struct FitState {
  char tag[8];          // "HMLEFIT1" once written
  int32_t dims, profile, iters, evals, failed;
  uint32_t fp;          // fingerprint of the data and the objective's options (fit_fingerprint)
  double n, best;
  hmle_theta best_th;
  double X[5][4], F[5], Q[5];
};
static_assert(sizeof(FitState) == HMLE_FIT_STATE_BYTES, "checkpoint layout");
constexpr char kStateTag[8] = {'H', 'M', 'L', 'E', 'F', 'I', 'T', '1'};

template <typename E>
hmle_status nelder_mead(E& f, const hmle_theta* start, const hmle_fit_opts& o, hmle_theta* theta_hat,
                        hmle_fit_report* report, std::chrono::steady_clock::time_point t0,
                        const FitState* resume = nullptr, FitState* save = nullptr) {
  // profiled fit: coordinate 0 is not searched, coordinate 3 codes the ratio
  // r = tau^2 / sigma^2 of the start
  const bool prof = f.obj.profile;
  const int D = prof ? 3 : 4, c0 = prof ? 1 : 0;
  std::array<Vec, 5> X{};
  std::array<double, 5> F{};
  int iters = 0;
  if (resume) {
    for (int i = 0; i <= D; ++i) {
      for (int d = 0; d < 4; ++d) X[i][d] = resume->X[i][d];
      F[i] = resume->F[i];
      if (std::isfinite(resume->Q[i])) f.quad.push_back({X[i], resume->Q[i]});
    }
    iters = resume->iters;
    f.evals = resume->evals;
    f.failed = resume->failed;
    f.best = resume->best;
    f.best_th = resume->best_th;
  } else {
    Vec x0 = start ? from_theta(*start) : Vec{2.0, 2.0, 1.0, 15.0};
    if (prof) {
      const hmle_theta th0 = to_theta(x0);
      x0[0] = 0.0;
      x0[3] = th0.tau2 > 0 ? -std::log(std::sqrt(th0.tau2 / th0.sigma2)) / std::log(2.0) : 60.0;
    }
    for (double v : x0)
      if (!std::isfinite(v)) return HMLE_E_INVALID;
    f.expect(nullptr, 0);
    double f0 = f(x0);
    if (o.use_backoff) {
      for (int k = 0; k < 30 && !std::isfinite(f0) && f.hard == HMLE_OK; ++k) {
        x0[3] -= 1.0;
        f0 = f(x0);
      }
    }
    if (f.hard != HMLE_OK) return f.hard;
    X[0] = x0;
    F[0] = f0;
    for (int i = 0; i < D; ++i) {
      X[i + 1] = x0;
      X[i + 1][c0 + i] += o.step;
    }
    f.expect(&X[1], D);
    for (int i = 0; i < D; ++i) F[i + 1] = f(X[i + 1]);
  }
  bool converged = false;
  std::array<int, 5> idx;
  while (true) {
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.begin() + D + 1, [&](int a, int b) { return F[a] < F[b]; });
    std::array<Vec, 5> Xs{};
    std::array<double, 5> Fs{};
    for (int i = 0; i <= D; ++i) { Xs[i] = X[idx[i]]; Fs[i] = F[idx[i]]; }
    X = Xs;
    F = Fs;
    double size = 0.0;
    for (int i = 1; i <= D; ++i)
      for (int d = 0; d < 4; ++d) size = std::max(size, std::fabs(X[i][d] - X[0][d]));
    if (size < o.tol && std::isfinite(F[0])) { converged = true; break; }
    if (iters >= o.max_iter) break;
    if (f.hard != HMLE_OK) break;
    ++iters;
    Vec c{0, 0, 0, 0};
    for (int i = 0; i < D; ++i)
      for (int d = 0; d < 4; ++d) c[d] += X[i][d] / double(D);
    auto lin = [&](double t, const Vec& a) {   // c + t (a - c)
      Vec r;
      for (int d = 0; d < 4; ++d) r[d] = c[d] + t * (a[d] - c[d]);
      return r;
    };
    const Vec xr = lin(-1.0, X[D]);
    const Vec xic = lin(0.5, X[D]), xoc = lin(-0.5, X[D]), xe = lin(-2.0, X[D]);
    const Vec cand[4] = {xr, xic, xoc, xe};
    f.expect(cand, 4);
    const double fr = f(xr);
    if (fr < F[0]) {
      const double fe = f(xe);
      if (fe < fr) { X[D] = xe; F[D] = fe; } else { X[D] = xr; F[D] = fr; }
      continue;
    }
    if (fr < F[D - 1]) { X[D] = xr; F[D] = fr; continue; }
    bool shrink = false;
    if (fr < F[D]) {
      const double fc = f(xoc);
      if (fc <= fr) { X[D] = xoc; F[D] = fc; } else shrink = true;
    } else {
      const double fc = f(xic);
      if (fc < F[D]) { X[D] = xic; F[D] = fc; } else shrink = true;
    }
    if (shrink) {
      for (int i = 1; i <= D; ++i)
        for (int d = 0; d < 4; ++d) X[i][d] = X[0][d] + 0.5 * (X[i][d] - X[0][d]);
      f.expect(&X[1], D);
      for (int i = 1; i <= D; ++i) F[i] = f(X[i]);
    }
  }
  if (f.hard != HMLE_OK) return f.hard;
  if (save) {
    *save = FitState{};
    std::memcpy(save->tag, kStateTag, sizeof kStateTag);
    save->dims = D;
    save->profile = prof ? 1 : 0;
    save->iters = iters;
    save->evals = f.evals;
    save->failed = f.failed;
    save->n = f.obj.n;
    save->best = f.best;
    save->best_th = f.best_th;
    for (int i = 0; i < 5; ++i) {
      for (int d = 0; d < 4; ++d) save->X[i][d] = X[i][d];
      save->F[i] = i <= D ? F[i] : INFINITY;
      save->Q[i] = i <= D ? f.quad_of(X[i]) : NAN;
    }
  }
  *theta_hat = to_theta(X[0]);
  if (prof) {
    // the variance that maximises eq. (1) at the best vertex
    const hmle_theta t = f.obj.point(X[0]);
    const double s2 = f.quad_of(X[0]) / f.obj.n;
    *theta_hat = hmle_theta{s2, t.range, t.nu, t.tau2 * s2};
  }
  if (report) {
    report->evals = f.evals;
    report->iters = iters;
    report->failed_evals = f.failed;
    report->converged = converged ? 1 : 0;
    report->logL = -F[0];
    report->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return converged ? HMLE_OK : HMLE_E_NOCONV;
}

bool read_opts(const hmle_fit_opts* opts, hmle_fit_opts& o) {
  hmle_default_fit_opts(&o);
  if (opts) o = *opts;
  return o.max_iter >= 1 && o.tol > 0 && o.step > 0;
}

}  // namespace

extern "C" hmle_status hmle_fit(hmle_problem p, const double* z, const hmle_theta* start, const hmle_fit_opts* opts,
                                hmle_theta* theta_hat, hmle_fit_report* report) {
  if (!p || !z || !theta_hat) return HMLE_E_INVALID;
  hmle_fit_opts o;
  if (!read_opts(opts, o)) return HMLE_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  SingleEval f;
  f.p = p;
  f.z = z;
  f.report_every = o.report_every;
  int64_t sz[6];
  if (hmle_sizes(p, sz) != HMLE_OK) return HMLE_E_INVALID;
  f.obj.profile = o.profile_variance != 0;
  f.obj.n = double(sz[0]);
  return nelder_mead(f, start, o, theta_hat, report, t0);
}

extern "C" hmle_status hmle_fit_resumable(hmle_problem p, const double* z, const hmle_theta* start,
                                          const hmle_fit_opts* opts, void* state, int64_t state_len,
                                          hmle_theta* theta_hat, hmle_fit_report* report) {
  if (!p || !z || !theta_hat || !state || state_len != (int64_t)sizeof(FitState)) return HMLE_E_INVALID;
  hmle_fit_opts o;
  if (!read_opts(opts, o)) return HMLE_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  SingleEval f;
  f.p = p;
  f.z = z;
  f.report_every = o.report_every;
  int64_t sz[6];
  if (hmle_sizes(p, sz) != HMLE_OK) return HMLE_E_INVALID;
  f.obj.profile = o.profile_variance != 0;
  f.obj.n = double(sz[0]);
  FitState in;
  std::memcpy(&in, state, sizeof in);
  const bool resume = std::memcmp(in.tag, kStateTag, sizeof kStateTag) == 0;
  // a checkpoint of another kind of search or of another problem size is refused
  if (resume && (in.dims != (f.obj.profile ? 3 : 4) || in.profile != (f.obj.profile ? 1 : 0) || in.n != f.obj.n ||
                 in.iters < 0 || in.evals < 0 || in.failed < 0 || in.failed > in.evals))
    return HMLE_E_INVALID;
  // and so is one of other data or other accuracy options
  uint32_t fp = 0;
  const hmle_status fs = hmle::fit_fingerprint(p, z, &fp);
  if (fs != HMLE_OK) return fs;
  if (resume && in.fp != fp) return HMLE_E_INVALID;
  FitState out;
  const hmle_status s = nelder_mead(f, start, o, theta_hat, report, t0, resume ? &in : nullptr, &out);
  out.fp = fp;
  if (s == HMLE_OK || s == HMLE_E_NOCONV) std::memcpy(state, &out, sizeof out);
  return s;
}

extern "C" hmle_status hmle_fit_batch(hmle_problem batch, const double* z, const hmle_theta* start,
                                      const hmle_fit_opts* opts, hmle_theta* theta_hat, hmle_fit_report* report,
                                      int32_t* rounds) {
  if (!batch || !z || !theta_hat) return HMLE_E_INVALID;
  hmle_fit_opts o;
  if (!read_opts(opts, o)) return HMLE_E_INVALID;
  const auto t0 = std::chrono::steady_clock::now();
  int32_t count = 0;
  int64_t n1 = 0;
  const hmle_status ls = hmle::candidate_layout(batch, &count, &n1);
  if (ls != HMLE_OK) return ls;
  double* zz = nullptr;
  hmle_status s = hmle::candidate_data(batch, z, count, n1, &zz);
  if (s == HMLE_OK) {
    BatchEval f;
    f.p = batch;
    f.zz = zz;
    f.count = count;
    f.report_every = o.report_every;
    f.obj.profile = o.profile_variance != 0;
    f.obj.n = double(n1);
    s = nelder_mead(f, start, o, theta_hat, report, t0);
    if (rounds) *rounds = f.rounds;
  }
  return s;
}
