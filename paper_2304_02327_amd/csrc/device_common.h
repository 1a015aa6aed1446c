// Device helpers: a complex-double type and the nonlinearities g(u).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/expint.h"

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

}  // namespace expint
