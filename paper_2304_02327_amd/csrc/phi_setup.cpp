// Host FP64 construction of the small matrices phi_l(tau A) of one direction.
//
// Definitions: paper section 1, eqs. integraldef / seriesdef.
// Construction (section 3.1): scale X = tau A by 2^s so that the scaled matrix
// is small, evaluate phi_0..phi_L of the scaled matrix, then undo the scaling
// with s steps of the squaring recurrence eq. squarephi
//     phi_l(2Y) = 2^{-l} [ e^Y phi_l(Y) + sum_{k=1}^{l} phi_k(Y) / (l-k)! ],
//     e^{2Y}    = e^Y e^Y.
// Where the paper evaluates the scaled phi_l with a Gauss-Lobatto quadrature
// of eq. integraldef, this code uses the Taylor series eq. seriesdef (Horner
// for the highest l, then phi_{l-1}(Y) = Y phi_l(Y) + I/(l-1)!), which for
// ||Y||_1 <= 1/2 and the degree chosen below is accurate to FP64 rounding.

#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.h"

namespace expint {
namespace {

using cplx = std::complex<double>;
thread_local bool t_single_threaded = false;

inline double absval(double x) { return std::fabs(x); }
inline double absval(const cplx& x) { return std::abs(x); }
inline bool finite(double x) { return std::isfinite(x); }
inline bool finite(const cplx& x) { return std::isfinite(x.real()) && std::isfinite(x.imag()); }

// C = A * B for n x n column-major matrices.  Columns of C are split over a
// few host threads; each column is computed by one thread in a fixed order,
// so the result does not depend on the thread count.
template <typename T>
void matmul(int n, const T* A, const T* B, T* C) {
  auto cols = [&](int j0, int j1) {
    const int KB = 64;
    for (int j = j0; j < j1; ++j) {
      T* c = C + (size_t)n * j;
      for (int i = 0; i < n; ++i) c[i] = T(0);
      for (int k0 = 0; k0 < n; k0 += KB) {
        const int k1 = k0 + KB < n ? k0 + KB : n;
        for (int k = k0; k < k1; ++k) {
          const T b = B[k + (size_t)n * j];
          const T* a = A + (size_t)n * k;
          for (int i = 0; i < n; ++i) c[i] += a[i] * b;
        }
      }
    }
  };
  const double work = double(n) * n * n;
  unsigned nt = 1;
  if (work > 2.0e6 && !t_single_threaded) {
    nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 16) nt = 16;
    if ((int)nt > n) nt = (unsigned)n;
  }
  if (nt <= 1) {
    cols(0, n);
    return;
  }
  std::vector<std::thread> pool;
  const int per = (n + (int)nt - 1) / (int)nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int j0 = (int)t * per, j1 = j0 + per < n ? j0 + per : n;
    if (j0 >= j1) break;
    pool.emplace_back(cols, j0, j1);
  }
  for (auto& th : pool) th.join();
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

template <typename T>
int phi_setup_impl(int n, const T* A, int lda, double tau, int ell_max, T* out, int ldo) {
  if (n < 1 || lda < n || ldo < n || !A || !out || ell_max < 0 || ell_max > 3)
    return set_error(EXPINT_EINVAL, "phi_setup: need n >= 1, lda >= n, ldphi >= n, non-NULL A/phi_out, 0 <= ell_max <= 3");
  if (!std::isfinite(tau)) return set_error(EXPINT_ENUMERIC, "phi_setup: tau is not finite");
  const size_t nn = (size_t)n * n;
  std::vector<T> X(nn);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const T a = A[i + (size_t)lda * j];
      if (!finite(a)) return set_error(EXPINT_ENUMERIC, "phi_setup: A has a non-finite entry");
      X[i + (size_t)n * j] = a * tau;
    }
  // scaling: ||X / 2^s||_1 <= 1/2
  double norm1 = 0.0;
  for (int j = 0; j < n; ++j) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += absval(X[i + (size_t)n * j]);
    norm1 = cs > norm1 ? cs : norm1;
  }
  int s = 0;
  while (norm1 > 0.5 && s < 1000) {
    norm1 *= 0.5;
    ++s;
  }
  const double scale = std::ldexp(1.0, -s);
  for (auto& x : X) x *= scale;
  // Taylor degree m: the first neglected term theta^{m+1}/(m+1)! below 1e-20
  int m = 4;
  while (m < 40 && std::pow(norm1, m + 1) / factorial(m + 1) > 1e-20) ++m;

  const int L = ell_max;
  std::vector<std::vector<T>> P(L + 1, std::vector<T>(nn));
  std::vector<T> tmp(nn);
  // Horner for phi_L(Y) = sum_{i=0}^{m} Y^i / (i+L)!
  std::vector<T>& PL = P[L];
  std::fill(PL.begin(), PL.end(), T(0));
  for (int i = 0; i < n; ++i) PL[i + (size_t)n * i] = T(1.0 / factorial(m + L));
  for (int i = m - 1; i >= 0; --i) {
    matmul(n, X.data(), PL.data(), tmp.data());
    const double c = 1.0 / factorial(i + L);
    for (int k = 0; k < n; ++k) tmp[k + (size_t)n * k] += T(c);
    PL.swap(tmp);
  }
  // phi_{l-1}(Y) = Y phi_l(Y) + I/(l-1)!
  for (int l = L; l >= 1; --l) {
    matmul(n, X.data(), P[l].data(), P[l - 1].data());
    const double c = 1.0 / factorial(l - 1);
    for (int k = 0; k < n; ++k) P[l - 1][k + (size_t)n * k] += T(c);
  }
  // s squaring steps (eq. squarephi), all from the previous values
  std::vector<std::vector<T>> Q(L + 1, std::vector<T>(nn));
  for (int step = 0; step < s; ++step) {
    for (int l = 0; l <= L; ++l) matmul(n, P[0].data(), P[l].data(), Q[l].data());
    for (int l = 1; l <= L; ++l) {
      const double w = std::ldexp(1.0, -l);
      for (size_t e = 0; e < nn; ++e) {
        T acc = Q[l][e];
        for (int k = 1; k <= l; ++k) acc += P[k][e] * T(1.0 / factorial(l - k));
        Q[l][e] = acc * w;
      }
    }
    P.swap(Q);
  }
  for (int l = 0; l <= L; ++l)
    for (int j = 0; j < n; ++j)
      std::memcpy(out + (size_t)l * ldo * n + (size_t)ldo * j, P[l].data() + (size_t)n * j, sizeof(T) * n);
  return EXPINT_OK;
}

}  // namespace

void phi_setup_single_threaded(bool on) { t_single_threaded = on; }

int phi_setup_real(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo) {
  return phi_setup_impl<double>(n, A, lda, tau, ell_max, out, ldo);
}

int phi_setup_complex(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo) {
  return phi_setup_impl<cplx>(n, reinterpret_cast<const cplx*>(A), lda, tau, ell_max,
                              reinterpret_cast<cplx*>(out), ldo);
}

}  // namespace expint
