// Matern covariance on the device, Section 1, eq. (2):
//
//   M(h) = sigma^2 * 2^(1-nu) / Gamma(nu) * x^nu K_nu(x),   x = h / ell,   M(0) = sigma^2.
//
// No library provides K_nu on the device, so it is computed here from
// published mathematics:
//   * half-integer orders nu = 1/2, 3/2, 5/2 use the elementary closed forms
//     of K_{n+1/2} (DLMF 10.39.2 and 10.29.1): M = sigma^2 e^{-x} p(x) with
//     p = 1, 1 + x, 1 + x + x^2/3;
//   * any other order: write nu = mu + m with |mu| <= 1/2 and evaluate
//     g_a(x) = x^a K_a(x) for a = mu and a = mu + 1 from the integral
//     representation K_a(x) = int_0^inf exp(-x cosh t) cosh(a t) dt
//     (DLMF 10.32.9) by the trapezoidal rule, whose error decays
//     exponentially in 1/step for this analytic, doubly-exponentially
//     decaying integrand; the step shrinks like 1/sqrt(x) for large x, where
//     the integrand is a narrow peak at t = 0. Then climb with the forward
//     recurrence K_{a+1} = K_{a-1} + (2a/x) K_a (DLMF 10.29.1), stable for
//     K, in the scaled form g_{a+1} = x^2 g_{a-1} + 2a g_a, which keeps every
//     quantity bounded by its value at x = 0, 2^(a-1) Gamma(a).
// exp, log and sqrt are the device library's.
#pragma once
#include "common.hpp"

namespace hmle {

template <typename T> struct KnuConst;
template <> struct KnuConst<double> {
  static constexpr double hmax = 0.25, hscale = 0.6, tol = 1e-17, xmax = 705.0;
};
template <> struct KnuConst<float> {
  static constexpr float hmax = 0.35f, hscale = 1.0f, tol = 1e-8f, xmax = 100.0f;
};

// g_mu(x) = x^mu K_mu(x) and g_{mu+1}(x) for |mu| <= 1/2, x > 0.
template <typename T>
__device__ __forceinline__ void knu_pair(T x, T mu, T& g0, T& g1) {
  using C = KnuConst<T>;
  const T a0 = mu < T(0) ? -mu : mu;
  const T a1 = mu + T(1);
  T hs = C::hscale / sqrt(x);
  if (hs > C::hmax) hs = C::hmax;
  const T e0 = exp(-x);
  T s0 = T(0.5) * e0, s1 = T(0.5) * e0;
  const T eh = exp(hs), ehi = T(1) / eh;
  const T ea0 = exp(a0 * hs), ea0i = T(1) / ea0;
  const T ea1 = exp(a1 * hs), ea1i = T(1) / ea1;
  T E = T(1), Ei = T(1), A0 = T(1), A0i = T(1), A1 = T(1), A1i = T(1);
  for (int k = 1; k < 400; ++k) {
    E *= eh; Ei *= ehi; A0 *= ea0; A0i *= ea0i; A1 *= ea1; A1i *= ea1i;
    const T ch = T(0.5) * (E + Ei);
    const T e = exp(-x * ch);
    const T t1 = e * (T(0.5) * (A1 + A1i));
    s0 += e * (T(0.5) * (A0 + A0i));
    s1 += t1;
    if (t1 <= C::tol * s1) break;
  }
  const T lx = log(x);
  g0 = exp(mu * lx) * (hs * s0);
  g1 = exp(a1 * lx) * (hs * s1);
}

// Matern value at distance h >= 0 (no nugget).
template <typename T>
__device__ __forceinline__ T matern_value(T h, const MaternParams& p) {
  if (h <= T(0)) return T(p.sigma2);
  const T x = h * T(p.inv_ell);
  if (x > KnuConst<T>::xmax) return T(0);
  if (p.kind == 0) return T(p.sigma2) * exp(-x);
  if (p.kind == 1) return T(p.sigma2) * (T(1) + x) * exp(-x);
  if (p.kind == 2) return T(p.sigma2) * (T(1) + x + x * x * T(1.0 / 3.0)) * exp(-x);
  T g0, g1;
  knu_pair<T>(x, T(p.mu), g0, g1);
  T g = g0;
  if (p.m >= 1) {
    g = g1;
    T a = T(p.mu) + T(1);
    const T x2 = x * x;
    for (int i = 1; i < p.m; ++i) {
      const T gn = x2 * g0 + T(2) * a * g1;
      g0 = g1;
      g1 = gn;
      a += T(1);
    }
    g = g1;
  }
  return T(p.pref) * g;
}

}  // namespace hmle
