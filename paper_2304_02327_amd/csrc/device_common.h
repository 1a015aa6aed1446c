// Device helpers: a complex-double type and the nonlinearities g(u).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/expint.h"
#include "internal.h"

namespace expint {

// interleaved complex double, 16-byte aligned like a pair of doubles in memory
struct __attribute__((aligned(16))) cdouble {
  double re, im;
};

template <typename T>
__device__ __forceinline__ T zero();
template <>
__device__ __forceinline__ double zero<double>() { return 0.0; }
template <>
__device__ __forceinline__ cdouble zero<cdouble>() { return cdouble{0.0, 0.0}; }

template <typename T>
__device__ __forceinline__ T real_value(double c);
template <>
__device__ __forceinline__ double real_value<double>(double c) { return c; }
template <>
__device__ __forceinline__ cdouble real_value<cdouble>(double c) { return cdouble{c, 0.0}; }

__device__ __forceinline__ double add(double a, double b) { return a + b; }
__device__ __forceinline__ cdouble add(cdouble a, cdouble b) { return cdouble{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ double sub(double a, double b) { return a - b; }
__device__ __forceinline__ cdouble sub(cdouble a, cdouble b) { return cdouble{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double scale(double a, double s) { return a * s; }
__device__ __forceinline__ cdouble scale(cdouble a, double s) { return cdouble{a.re * s, a.im * s}; }
// c * x + acc
__device__ __forceinline__ double fma_t(double c, double x, double acc) { return fma(c, x, acc); }
__device__ __forceinline__ cdouble fma_t(cdouble c, cdouble x, cdouble acc) {
  return cdouble{fma(c.re, x.re, fma(-c.im, x.im, acc.re)), fma(c.re, x.im, fma(c.im, x.re, acc.im))};
}

// Manufactured-solution nonlinearity of the paper's advection-diffusion-
// reaction test (section 4.2, eq. ADR): g = 1/(1 + u^2) + Psi(t, x) with Psi
// such that u = e^t 64 prod_mu x_mu (1 - x_mu) solves
// u_t = eps Laplace(u) + alpha sum_mu d_mu u + g.  With q = x (1 - x), q' = 1 - 2x,
// q'' = -2:  Psi = u - eps e^t 64 sum_mu q''_mu prod_{nu != mu} q_nu
//                 - alpha e^t 64 sum_mu q'_mu prod_{nu != mu} q_nu - 1/(1 + u^2).
// x_mu = (i_mu + 1) h_mu on the inner grid, h_mu = 1/(n_mu + 1).

// Psi part of the source with E = 64 e^t precomputed (t is uniform per launch).
__device__ __forceinline__ double adr_paper_g_E(const GridTime& c, double E, double u, int i1, int i2, int i3) {
  const double x1 = (i1 + 1) * c.h[0], x2 = (i2 + 1) * c.h[1], x3 = (i3 + 1) * c.h[2];
  const double q1 = x1 * (1.0 - x1), q2 = x2 * (1.0 - x2), q3 = x3 * (1.0 - x3);
  const double d1 = 1.0 - 2.0 * x1, d2 = 1.0 - 2.0 * x2, d3 = 1.0 - 2.0 * x3;
  const double ue = E * q1 * q2 * q3;
  const double lap = E * (-2.0) * (q2 * q3 + q1 * q3 + q1 * q2);
  const double adv = E * (d1 * q2 * q3 + q1 * d2 * q3 + q1 * q2 * d3);
  const double psi = ue - c.eps * lap - c.alpha * adv - 1.0 / (1.0 + ue * ue);
  return 1.0 / (1.0 + u * u) + psi;
}

__device__ __forceinline__ double adr_paper_g(const GridTime& c, double u, double t, int i1, int i2, int i3) {
  return adr_paper_g_E(c, 64.0 * exp(t), u, i1, i2, i3);
}

__device__ __forceinline__ double clock_time(const GridTime& c, double ahead) {
  return c.clock[0] + c.clock[1] * c.tau + ahead;
}

// g at tensor element e (layout i1 + n1 (i2 + n2 i3)), time t_n + ahead
__device__ __forceinline__ double g_at(int g, double u, double gparam, const GridTime& gt, long e, double ahead) {
  if (g == EXPINT_G_ADR_PAPER) {
    const int i1 = (int)(e % gt.n[0]);
    const long r = e / gt.n[0];
    const int i2 = (int)(r % gt.n[1]);
    const int i3 = (int)(r / gt.n[1]);
    return adr_paper_g(gt, u, clock_time(gt, ahead), i1, i2, i3);
  }
  switch (g) {
    case EXPINT_G_ALLEN_CAHN:
      return u - u * u * u;
    case EXPINT_G_U2_1MU:
      return u * u * (1.0 - u);
    default:
      return 0.0;
  }
}
__device__ __forceinline__ cdouble g_at(int g, cdouble u, double gparam, const GridTime&, long, double) {
  if (g == EXPINT_G_CUBIC_NLS) {
    const double m = gparam * (u.re * u.re + u.im * u.im);
    return cdouble{m * u.im, -m * u.re};
  }
  return cdouble{0.0, 0.0};
}

// g(u) for the autonomous nonlinearities of the workloads
__device__ __forceinline__ double g_eval(int g, double u, double /*p*/) {
  switch (g) {
    case EXPINT_G_ALLEN_CAHN:
      return u - u * u * u;
    case EXPINT_G_U2_1MU:
      return u * u * (1.0 - u);
    default:
      return 0.0;
  }
}

// complex: g = -i kappa |u|^2 u  ->  (kappa |u|^2 im, -kappa |u|^2 re)
__device__ __forceinline__ cdouble g_eval(int g, cdouble u, double kappa) {
  if (g == EXPINT_G_CUBIC_NLS) {
    const double m = kappa * (u.re * u.re + u.im * u.im);
    return cdouble{m * u.im, -m * u.re};
  }
  return cdouble{0.0, 0.0};
}

// Per-launch evaluators of g for kernels that apply g to many elements with
// the op and the nonlinearity fixed for the whole launch: at(ahead) does the
// time-dependent work once for t = t_n + ahead, and the returned object
// evaluates g(t, u) at tensor element e.  dispatch_g picks the evaluator from
// the epilogue's nonlinearity code, so that a kernel instantiates one compact
// loop per nonlinearity instead of a per-element switch.
struct GZero {
  __device__ __forceinline__ GZero at(double) const { return *this; }
  template <typename T>
  __device__ __forceinline__ T operator()(T, long) const { return zero<T>(); }
};
struct GAllenCahn {
  __device__ __forceinline__ GAllenCahn at(double) const { return *this; }
  __device__ __forceinline__ double operator()(double u, long) const { return u - u * u * u; }
};
struct GU21mu {
  __device__ __forceinline__ GU21mu at(double) const { return *this; }
  __device__ __forceinline__ double operator()(double u, long) const { return u * u * (1.0 - u); }
};
struct GCubicNls {
  double kappa;
  __device__ __forceinline__ GCubicNls at(double) const { return *this; }
  __device__ __forceinline__ cdouble operator()(cdouble u, long) const {
    const double m = kappa * (u.re * u.re + u.im * u.im);
    return cdouble{m * u.im, -m * u.re};
  }
};
// Element e = i1 + n1 (i2 + n2 i3) of a tensor below 2^31 elements (the
// library caps tensors at 2 GiB), so 32-bit index arithmetic is exact.
struct GAdrPaper {
  GridTime c;
  double E;
  __device__ __forceinline__ GAdrPaper at(double ahead) const {
    GAdrPaper r = *this;
    r.E = 64.0 * exp(clock_time(c, ahead));
    return r;
  }
  __device__ __forceinline__ double operator()(double u, long e) const {
    const unsigned n0 = (unsigned)c.n[0], n1 = (unsigned)c.n[1];
    const unsigned ee = (unsigned)e, r = ee / n0;
    return adr_paper_g_E(c, E, u, (int)(ee - r * n0), (int)(r % n1), (int)(r / n1));
  }
};

template <typename F>
__device__ __forceinline__ void dispatch_g(const Epilogue& ep, double, F&& f) {
  switch (ep.g) {
    case EXPINT_G_ALLEN_CAHN:
      f(GAllenCahn{});
      break;
    case EXPINT_G_U2_1MU:
      f(GU21mu{});
      break;
    case EXPINT_G_ADR_PAPER:
      f(GAdrPaper{ep.gt, 0.0});
      break;
    default:
      f(GZero{});
      break;
  }
}
template <typename F>
__device__ __forceinline__ void dispatch_g(const Epilogue& ep, cdouble, F&& f) {
  if (ep.g == EXPINT_G_CUBIC_NLS)
    f(GCubicNls{ep.gparam});
  else
    f(GZero{});
}

}  // namespace expint
