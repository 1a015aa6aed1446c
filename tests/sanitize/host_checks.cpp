// Host driver for the sanitizer build of the library's host-only code (the phi
// construction and the argument checks): every call below must return the
// status it documents, and the address / undefined-behaviour sanitizers must
// report nothing.  Built and run by tests/test_sanitize_host.py with g++
// -fsanitize=address,undefined; it links phi_setup.cpp and host_abi.cpp only.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "expint.h"

static int g_fail = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                           \
    }                                                                     \
  } while (0)

// phi_l(0) = I / l!: the tau = 0 case of the construction
static void check_tau_zero(int n, int ell_max, int method, int dtype) {
  const int w = dtype == EXPINT_C128 ? 2 : 1;
  std::vector<double> A((size_t)n * n * w, 0.5), out((size_t)(ell_max + 1) * n * n * w, -1.0);
  EXPECT(phi_setup_ex(n, A.data(), n, 0.0, ell_max, method, dtype, out.data(), n) == EXPINT_OK);
  double fact = 1.0;
  for (int l = 0; l <= ell_max; ++l) {
    if (l > 0) fact *= l;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double want = i == j ? 1.0 / fact : 0.0;
        EXPECT(std::fabs(out[(((size_t)l * n + j) * n + i) * w] - want) <= 1e-15);
      }
  }
}

int main() {
  std::mt19937_64 rng(7);
  std::normal_distribution<double> N01(0.0, 1.0);
  // the constructions on random matrices of many sizes, scales, strides and phi orders
  for (int n : {1, 2, 3, 5, 8, 17, 33, 64, 97}) {
    for (double scale : {1e-3, 0.7, 40.0}) {
      const int lda = n + 3, ldphi = n + 1;
      std::vector<double> A((size_t)lda * n), Az((size_t)lda * n * 2);
      for (auto& x : A) x = scale * N01(rng) / std::sqrt((double)n);
      for (auto& x : Az) x = scale * N01(rng) / std::sqrt((double)n);
      for (int ell = 0; ell <= 3; ++ell) {
        std::vector<double> out((size_t)(ell + 1) * ldphi * n), outz((size_t)(ell + 1) * ldphi * n * 2);
        EXPECT(phi_setup(n, A.data(), lda, 0.3, ell, out.data(), ldphi) == EXPINT_OK);
        EXPECT(phi_setup_z(n, Az.data(), lda, 0.3, ell, outz.data(), ldphi) == EXPINT_OK);
        for (int method : {EXPINT_PHI_TAYLOR, EXPINT_PHI_QUAD}) {
          std::vector<double> o2((size_t)(ell + 1) * ldphi * n);
          EXPECT(phi_setup_ex(n, A.data(), lda, 0.3, ell, method, EXPINT_F64, o2.data(), ldphi) == EXPINT_OK);
          for (size_t k = 0; k < o2.size(); ++k) EXPECT(std::isfinite(o2[k]));
        }
        for (double v : out) EXPECT(std::isfinite(v));
      }
    }
  }
  for (int method : {EXPINT_PHI_TAYLOR, EXPINT_PHI_QUAD}) {
    check_tau_zero(6, 3, method, EXPINT_F64);
    check_tau_zero(5, 2, method, EXPINT_C128);
  }
  // rejected arguments: documented status, nothing written past the buffers
  {
    std::vector<double> A(16, 1.0), out(64, 0.0);
    EXPECT(phi_setup(0, A.data(), 4, 0.1, 1, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(phi_setup(4, nullptr, 4, 0.1, 1, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(phi_setup(4, A.data(), 3, 0.1, 1, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(phi_setup(4, A.data(), 4, 0.1, 1, out.data(), 3) == EXPINT_EINVAL);
    EXPECT(phi_setup(4, A.data(), 4, 0.1, 4, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(phi_setup(4, A.data(), 4, std::numeric_limits<double>::quiet_NaN(), 1, out.data(), 4) == EXPINT_ENUMERIC);
    A[5] = std::numeric_limits<double>::infinity();
    EXPECT(phi_setup(4, A.data(), 4, 0.1, 1, out.data(), 4) == EXPINT_ENUMERIC);
    EXPECT(phi_setup_ex(4, A.data(), 4, 0.1, 1, 7, EXPINT_F64, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(phi_setup_ex(4, A.data(), 4, 0.1, 1, EXPINT_PHI_QUAD, 9, out.data(), 4) == EXPINT_EINVAL);
    EXPECT(expint_last_error()[0] != '\0');
  }
  // workspace sizes and shape checks
  {
    size_t bytes = 0;
    const int ok3[3] = {40, 41, 130};
    for (int prec = 0; prec <= 3; ++prec) EXPECT(tucker_workspace_size(3, ok3, EXPINT_F64, prec, &bytes) == EXPINT_OK);
    EXPECT(tucker_workspace_size(3, ok3, EXPINT_C128, EXPINT_PREC_FP64, &bytes) == EXPINT_OK);
    const int zero[2] = {5, 0}, huge[3] = {2048, 2048, 1024}, d5[5] = {1, 1, 1, 1, 1};
    EXPECT(tucker_workspace_size(2, zero, EXPINT_F64, 0, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(3, huge, EXPINT_F64, 0, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(5, d5, EXPINT_F64, 0, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(0, d5, EXPINT_F64, 0, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(3, ok3, 5, 0, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(3, ok3, EXPINT_F64, 9, &bytes) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(3, ok3, EXPINT_F64, 0, nullptr) == EXPINT_EINVAL);
    EXPECT(tucker_workspace_size(3, nullptr, EXPINT_F64, 0, &bytes) == EXPINT_EINVAL);
  }
  std::printf("host checks: %d failures\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}
