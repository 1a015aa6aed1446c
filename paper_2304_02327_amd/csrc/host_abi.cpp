// C-ABI entry points that run on the host only (the phi construction, workspace
// sizes, the error message) and the argument checks the device entry points
// share.  Plain C++: this file and phi_setup.cpp also build on their own under
// the host address and undefined-behaviour sanitizers (tests/sanitize).
#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>

#include "internal.h"

namespace expint {

namespace {
thread_local char g_errbuf[512] = "";
}

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_errbuf, sizeof(g_errbuf), fmt, ap);
  va_end(ap);
  return code;
}

namespace {
size_t elem_size(int dtype) { return dtype == EXPINT_C128 ? 16 : 8; }
}  // namespace

int slice_kpad(int n) { return (n + 63) / 64 * 64; }

size_t slice_digits_bytes(long rows, int n) {
  const size_t plane = (size_t)rows * (size_t)slice_kpad(n);
  return ((size_t)kSliceDigits * plane + 255) / 256 * 256 + ((size_t)rows * sizeof(int) + 255) / 256 * 256;
}

// Bytes of the digit buffer of a sliced chain: the largest per-mode tensor digits.
size_t sliced_tensor_digits_bytes(int d, const int* n, long N) {
  size_t b = 0;
  for (int mu = 0; mu < d; ++mu) b = std::max(b, slice_digits_bytes(N / n[mu], n[mu]));
  return b;
}

bool valid_precision(int precision) {
  return precision == EXPINT_PREC_FP64 || precision == EXPINT_PREC_FP32 || precision == EXPINT_PREC_BF16X3 ||
         precision == EXPINT_PREC_SLICED;
}

#define TRY(expr)              \
  do {                         \
    int r_ = (expr);           \
    if (r_ != EXPINT_OK) return r_; \
  } while (0)

int validate_shape(int d, const int* n, long* N) {
  if (d < 1 || d > 4 || !n) return set_error(EXPINT_EINVAL, "need 1 <= d <= 4 and a size array");
  long tot = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1) return set_error(EXPINT_EINVAL, "n[%d] = %d must be >= 1", mu, n[mu]);
    tot *= n[mu];
    if (tot >= (1L << 31)) return set_error(EXPINT_EINVAL, "tensor too large (prod n >= 2^31)");
  }
  *N = tot;
  return EXPINT_OK;
}

// Operand limits of the kernels, checked before anything is enqueued: every
// mu-mode product addresses its operands with 32-bit buffer offsets (below
// 2 GiB per tensor), and the exact-slice digits need n_mu <= 26624 and each
// digit plane (fibres x padded length) below 2^31 bytes.
int check_operand_limits(int d, const int* n, long N, int dtype, int precision) {
  const size_t bytes = (size_t)N * elem_size(dtype);
  if (bytes >= (1ull << 31))
    return set_error(EXPINT_ENOTSUP, "a tensor of %zu bytes exceeds the 2 GiB limit of one mu-mode product operand",
                     bytes);
  if (precision == EXPINT_PREC_SLICED)
    for (int mu = 0; mu < d; ++mu) {
      if (n[mu] > kSliceMaxK)
        return set_error(EXPINT_ENOTSUP, "exact-slice precision: n[%d] = %d exceeds %d", mu, n[mu], kSliceMaxK);
      const size_t plane = (size_t)(N / n[mu]) * (size_t)slice_kpad(n[mu]);
      if (plane >= (1ull << 31))
        return set_error(EXPINT_ENOTSUP, "exact-slice precision: digit plane of mode %d exceeds 2 GiB", mu + 1);
    }
  return EXPINT_OK;
}

// Workspace layout of tucker_apply: FP64 / FP32 / BF16X3 use up to two
// ping-pong tensors of N elements; the exact-slice chain uses one FP64 tensor,
// the digit buffer of the largest mode and the digits of every M.
int tucker_ws_layout(int d, const int* n, long N, int dtype, int precision, int modes, size_t* tensors,
                            size_t* digits, size_t* mdigits) {
  *tensors = *digits = *mdigits = 0;
  if (precision == EXPINT_PREC_SLICED) {
    *tensors = modes > 1 ? ((size_t)N * 8 + 255) / 256 * 256 : 0;
    *digits = sliced_tensor_digits_bytes(d, n, N);
    for (int mu = 0; mu < d; ++mu) *mdigits += slice_digits_bytes(n[mu], n[mu]);
    return EXPINT_OK;
  }
  const int bufs = modes - 1 < 2 ? modes - 1 : 2;
  *tensors = (size_t)bufs * (size_t)N * elem_size(dtype);
  return EXPINT_OK;
}

}  // namespace expint

using namespace expint;

extern "C" int tucker_workspace_size(int d, const int* n, int dtype, int precision, size_t* bytes) {
  long N;
  TRY(validate_shape(d, n, &N));
  if (dtype != EXPINT_F64 && dtype != EXPINT_C128) return set_error(EXPINT_EINVAL, "unknown dtype %d", dtype);
  if (!valid_precision(precision)) return set_error(EXPINT_EINVAL, "unknown precision %d", precision);
  if (!bytes) return set_error(EXPINT_EINVAL, "bytes is NULL");
  size_t t, g, m;
  TRY(tucker_ws_layout(d, n, N, dtype, precision, d, &t, &g, &m));
  *bytes = t + g + m;
  return EXPINT_OK;
}

// ---------------------------------------------------------------------------
// phi_setup
// ---------------------------------------------------------------------------

extern "C" int phi_setup(int n, const double* A, int lda, double tau, int ell_max, double* phi_out,
                         int ldphi) {
  try {
    return phi_setup_real(n, A, lda, tau, ell_max, phi_out, ldphi);
  } catch (const std::bad_alloc&) {
    return set_error(EXPINT_ENOMEM, "phi_setup: out of host memory");
  }
}

extern "C" int phi_setup_z(int n, const double* A, int lda, double tau, int ell_max, double* phi_out,
                           int ldphi) {
  try {
    return phi_setup_complex(n, A, lda, tau, ell_max, phi_out, ldphi);
  } catch (const std::bad_alloc&) {
    return set_error(EXPINT_ENOMEM, "phi_setup_z: out of host memory");
  }
}

extern "C" int phi_setup_ex(int n, const double* A, int lda, double tau, int ell_max, int method, int dtype,
                            double* phi_out, int ldphi) {
  if (dtype != EXPINT_F64 && dtype != EXPINT_C128) return set_error(EXPINT_EINVAL, "phi_setup_ex: unknown dtype %d", dtype);
  try {
    return phi_setup_method(method, dtype == EXPINT_C128, n, A, lda, tau, ell_max, phi_out, ldphi);
  } catch (const std::bad_alloc&) {
    return set_error(EXPINT_ENOMEM, "phi_setup_ex: out of host memory");
  }
}

extern "C" const char* expint_last_error(void) { return g_errbuf; }

extern "C" const char* expint_version(void) { return "expint 0.1.0 (gfx950)"; }
