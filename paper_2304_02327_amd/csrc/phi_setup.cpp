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
using cplx_t = std::complex<double>;
namespace {

using cplx = std::complex<double>;
constexpr int kPhiQuadNodes = 8;  // Gauss-Legendre-Lobatto nodes of eq. phiquad
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
  int assigned = 0;  // columns [0, assigned) belong to started threads
  try {
    pool.reserve(nt);
    for (unsigned t = 0; t < nt; ++t) {
      const int j0 = (int)t * per, j1 = j0 + per < n ? j0 + per : n;
      if (j0 >= j1) break;
      pool.emplace_back(cols, j0, j1);
      assigned = j1;
    }
  } catch (...) {
    // no more threads: the calling thread computes the columns left over
  }
  cols(assigned, n);
  for (auto& th : pool) th.join();
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

template <typename T>
double norm_1(int n, const T* X) {
  double norm1 = 0.0;
  for (int j = 0; j < n; ++j) {
    double cs = 0.0;
    for (int i = 0; i < n; ++i) cs += absval(X[i + (size_t)n * j]);
    norm1 = cs > norm1 ? cs : norm1;
  }
  return norm1;
}

// X = tau A (n x n, from a column-major A with leading dimension lda), scaled
// by 2^-s with s the smallest count for which ||X / 2^s||_1 <= limit (strictly
// below when `strict`).  Returns the status; *s and *norm1 (the scaled norm)
// on success.
template <typename T>
int scaled_input(int n, const T* A, int lda, double tau, double limit, bool strict, std::vector<T>& X, int* s_out,
                 double* norm_out) {
  const size_t nn = (size_t)n * n;
  X.assign(nn, T(0));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const T a = A[i + (size_t)lda * j];
      if (!finite(a)) return set_error(EXPINT_ENUMERIC, "phi_setup: A has a non-finite entry");
      X[i + (size_t)n * j] = a * tau;
    }
  double norm1 = norm_1(n, X.data());
  int s = 0;
  while ((strict ? norm1 >= limit : norm1 > limit) && s < 1000) {
    norm1 *= 0.5;
    ++s;
  }
  const double scale = std::ldexp(1.0, -s);
  for (auto& x : X) x *= scale;
  *s_out = s;
  *norm_out = norm1;
  return EXPINT_OK;
}

// Undoes the scaling with s steps of eq. squarephi (every phi_l of the new
// step from the previous values, e^{2Y} = (e^Y)^2) and copies phi_0..phi_L out.
template <typename T>
void unscale_and_store(int n, int L, int s, std::vector<std::vector<T>>& P, T* out, int ldo) {
  const size_t nn = (size_t)n * n;
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
}

int check_phi_args(int n, const void* A, int lda, double tau, int ell_max, const void* out, int ldo) {
  if (n < 1 || lda < n || ldo < n || !A || !out || ell_max < 0 || ell_max > 3)
    return set_error(EXPINT_EINVAL, "phi_setup: need n >= 1, lda >= n, ldphi >= n, non-NULL A/phi_out, 0 <= ell_max <= 3");
  if (!std::isfinite(tau)) return set_error(EXPINT_ENUMERIC, "phi_setup: tau is not finite");
  return EXPINT_OK;
}

template <typename T>
int phi_setup_impl(int n, const T* A, int lda, double tau, int ell_max, T* out, int ldo) {
  if (int rc = check_phi_args(n, A, lda, tau, ell_max, out, ldo); rc != EXPINT_OK) return rc;
  const size_t nn = (size_t)n * n;
  std::vector<T> X;
  int s = 0;
  double norm1;
  if (int rc = scaled_input(n, A, lda, tau, 0.5, false, X, &s, &norm1); rc != EXPINT_OK)  // ||X / 2^s||_1 <= 1/2
    return rc;
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
  unscale_and_store(n, L, s, P, out, ldo);
  return EXPINT_OK;
}

// ---- the paper's construction: quadrature of eq. integraldef (section 3.1) ----

// Gauss-Legendre-Lobatto rule with q nodes on [0, 1]: the end points and the
// roots of P'_N (N = q - 1) mapped from [-1, 1], weights 1 / (N (N+1) P_N(x)^2)
// (half the weights on [-1, 1]).  Interior nodes are Newton iterates on
// f(x) = (1 - x^2) P'_N(x) = N (P_{N-1}(x) - x P_N(x)), f'(x) = -N (N+1) P_N(x),
// from the Chebyshev-Gauss-Lobatto points.
void gll_rule(int q, double* theta, double* w) {
  const int N = q - 1;
  auto legendre = [N](double x, double* pn, double* pn1) {  // P_N(x), P_{N-1}(x) by the three-term recurrence
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= N; ++k) {
      const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    *pn = p1;
    *pn1 = p0;
  };
  for (int k = 0; k <= N; ++k) {
    double x = -std::cos(M_PI * k / N);
    if (k > 0 && k < N)
      for (int it = 0; it < 100; ++it) {
        double pn, pn1;
        legendre(x, &pn, &pn1);
        const double dx = (pn1 - x * pn) / ((N + 1) * pn);
        x += dx;
        if (std::fabs(dx) < 1e-16) break;
      }
    double pn, pn1;
    legendre(x, &pn, &pn1);
    theta[k] = k == 0 ? 0.0 : (k == N ? 1.0 : 0.5 * (x + 1.0));
    w[k] = 1.0 / (N * (N + 1) * pn * pn);
  }
}

// X = B^{-1} C by Gaussian elimination with partial pivoting (n x n,
// column-major; B and C are overwritten, the solution is left in C).
template <typename T>
int solve_in_place(int n, std::vector<T>& B, std::vector<T>& C) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = absval(B[k + (size_t)n * k]);
    for (int i = k + 1; i < n; ++i)
      if (absval(B[i + (size_t)n * k]) > best) best = absval(B[i + (size_t)n * k]), p = i;
    if (!(best > 0.0)) return set_error(EXPINT_ENUMERIC, "phi_setup: singular Pade denominator");
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(B[k + (size_t)n * j], B[p + (size_t)n * j]);
      for (int j = 0; j < n; ++j) std::swap(C[k + (size_t)n * j], C[p + (size_t)n * j]);
    }
    const T inv = T(1.0) / B[k + (size_t)n * k];
    for (int i = k + 1; i < n; ++i) {
      const T f = B[i + (size_t)n * k] * inv;
      if (f == T(0)) continue;
      for (int j = k + 1; j < n; ++j) B[i + (size_t)n * j] -= f * B[k + (size_t)n * j];
      for (int j = 0; j < n; ++j) C[i + (size_t)n * j] -= f * C[k + (size_t)n * j];
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = n - 1; i >= 0; --i) {
      T acc = C[i + (size_t)n * j];
      for (int k = i + 1; k < n; ++k) acc -= B[i + (size_t)n * k] * C[k + (size_t)n * j];
      C[i + (size_t)n * j] = acc / B[i + (size_t)n * i];
    }
  return EXPINT_OK;
}

// e^Z by the diagonal [m/m] Pade approximant D_m(Z)^{-1} N_m(Z) with
// N_m(Z) = sum_j b_j Z^j, D_m(Z) = sum_j (-1)^j b_j Z^j,
// b_j = (2m - j)! m! / ((2m)! j! (m - j)!), m the smallest degree in
// {3, 5, 7, 9, 13} whose backward-error bound theta_m (Higham 2005, the method
// behind the paper's expm) covers ||Z||_1, and scaling and squaring beyond
// theta_13.
template <typename T>
int expm_pade(int n, const T* Z, T* out) {
  static const int kDeg[] = {3, 5, 7, 9, 13};
  static const double kTheta[] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1,
                                  2.097847961257068e0, 5.371920351148152e0};
  const size_t nn = (size_t)n * n;
  double nz = norm_1(n, Z);
  int sq = 0, m = 13;
  for (int i = 0; i < 5; ++i)
    if (nz <= kTheta[i]) {
      m = kDeg[i];
      break;
    }
  while (nz > kTheta[4]) {
    nz *= 0.5;
    ++sq;
  }
  std::vector<T> Zs(Z, Z + nn);
  const double sc = std::ldexp(1.0, -sq);
  for (auto& z : Zs) z *= sc;
  std::vector<T> Num(nn, T(0)), Den(nn, T(0)), Pw(nn), tmp(nn);
  for (int i = 0; i < n; ++i) Num[i + (size_t)n * i] = Den[i + (size_t)n * i] = T(1.0);  // b_0 = 1
  Pw = Zs;
  double b = 1.0;
  for (int j = 1; j <= m; ++j) {
    b *= double(m - j + 1) / (double(j) * double(2 * m - j + 1));  // b_j / b_{j-1}
    const double sd = (j % 2) ? -b : b;
    for (size_t e = 0; e < nn; ++e) {
      Num[e] += Pw[e] * T(b);
      Den[e] += Pw[e] * T(sd);
    }
    if (j < m) {
      matmul(n, Zs.data(), Pw.data(), tmp.data());
      Pw.swap(tmp);
    }
  }
  if (int rc = solve_in_place(n, Den, Num); rc != EXPINT_OK) return rc;
  for (int k = 0; k < sq; ++k) {
    matmul(n, Num.data(), Num.data(), tmp.data());
    Num.swap(tmp);
  }
  std::memcpy(out, Num.data(), sizeof(T) * nn);
  return EXPINT_OK;
}

// The paper's phi builder: scale X = tau A by 2^s with ||X / 2^s||_1 < 1,
// phi_0(Y) = e^Y and, for l > 0, phi_l(Y) ~ sum_i w_i e^{(1-theta_i) Y}
// theta_i^{l-1} / (l-1)! on the Gauss-Legendre-Lobatto rule (eq. phiquad; the
// node theta = 0 gives e^Y itself, the node theta = 1 the identity), then the
// squaring recurrence eq. squarephi.
template <typename T>
int phi_setup_quad_impl(int n, const T* A, int lda, double tau, int ell_max, T* out, int ldo) {
  if (int rc = check_phi_args(n, A, lda, tau, ell_max, out, ldo); rc != EXPINT_OK) return rc;
  const size_t nn = (size_t)n * n;
  std::vector<T> X;
  int s = 0;
  double norm1;
  if (int rc = scaled_input(n, A, lda, tau, 1.0, true, X, &s, &norm1); rc != EXPINT_OK) return rc;
  const int L = ell_max;
  std::vector<std::vector<T>> P(L + 1, std::vector<T>(nn, T(0)));
  if (L == 0) {
    if (int rc = expm_pade(n, X.data(), P[0].data()); rc != EXPINT_OK) return rc;
  } else {
    double theta[kPhiQuadNodes], w[kPhiQuadNodes];
    gll_rule(kPhiQuadNodes, theta, w);
    std::vector<T> E(nn), Z(nn);
    for (int i = 0; i < kPhiQuadNodes; ++i) {
      if (i == kPhiQuadNodes - 1) {
        std::fill(E.begin(), E.end(), T(0));
        for (int k = 0; k < n; ++k) E[k + (size_t)n * k] = T(1.0);
      } else {
        for (size_t e = 0; e < nn; ++e) Z[e] = X[e] * (1.0 - theta[i]);
        if (int rc = expm_pade(n, Z.data(), E.data()); rc != EXPINT_OK) return rc;
      }
      if (i == 0) P[0] = E;
      for (int l = 1; l <= L; ++l) {
        const double c = w[i] * std::pow(theta[i], l - 1) / factorial(l - 1);
        if (c == 0.0) continue;
        for (size_t e = 0; e < nn; ++e) P[l][e] += E[e] * c;
      }
    }
  }
  unscale_and_store(n, L, s, P, out, ldo);
  return EXPINT_OK;
}

}  // namespace

void phi_setup_single_threaded(bool on) { t_single_threaded = on; }

int phi_setup_method(int method, bool cplx, int n, const double* A, int lda, double tau, int ell_max, double* out,
                     int ldo) {
  if (method == EXPINT_PHI_TAYLOR)
    return cplx ? phi_setup_impl<cplx_t>(n, reinterpret_cast<const cplx_t*>(A), lda, tau, ell_max,
                                         reinterpret_cast<cplx_t*>(out), ldo)
                : phi_setup_impl<double>(n, A, lda, tau, ell_max, out, ldo);
  if (method == EXPINT_PHI_QUAD)
    return cplx ? phi_setup_quad_impl<cplx_t>(n, reinterpret_cast<const cplx_t*>(A), lda, tau, ell_max,
                                              reinterpret_cast<cplx_t*>(out), ldo)
                : phi_setup_quad_impl<double>(n, A, lda, tau, ell_max, out, ldo);
  return set_error(EXPINT_EINVAL, "phi_setup: unknown method %d", method);
}

int phi_setup_real(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo) {
  return phi_setup_impl<double>(n, A, lda, tau, ell_max, out, ldo);
}

int phi_setup_complex(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo) {
  return phi_setup_impl<cplx>(n, reinterpret_cast<const cplx*>(A), lda, tau, ell_max,
                              reinterpret_cast<cplx*>(out), ldo);
}

}  // namespace expint
