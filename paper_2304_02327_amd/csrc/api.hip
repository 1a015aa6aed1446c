// C ABI: argument validation, plans and the per-step kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace expint {


namespace {

size_t elem_size(int dtype) { return dtype == EXPINT_C128 ? 16 : 8; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return set_error(EXPINT_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int r_ = (expr);           \
    if (r_ != EXPINT_OK) return r_; \
  } while (0)

// Tensor view of mode mu (0-based) of a d-tensor: (s, n_mu, r)
void mode_view(int d, const int* n, int mu, long* s, long* r) {
  long a = 1, b = 1;
  for (int k = 0; k < mu; ++k) a *= n[k];
  for (int k = mu + 1; k < d; ++k) b *= n[k];
  *s = a;
  *r = b;
}

// Modes 1 and 2 run as one launch (FP64 real data, n2 <= 128) unless
// EXPINT_FUSE12=0, EXPINT_TILE forces a single-mode tile on every mode, or the
// autotuner (or EXPINT_M12=off) found the two single-mode launches faster.
bool fuse12_allowed(int dtype, int precision, int d, const int* n) {
  const char* fenv = std::getenv("EXPINT_FUSE12");
  if (!(precision == EXPINT_PREC_FP64 && dtype == EXPINT_F64 && d >= 2 && modes12_fits(n[0], n[1]) &&
        !(fenv && fenv[0] == '0') && !std::getenv("EXPINT_TILE")))
    return false;
  long r = 1;
  for (int k = 2; k < d; ++k) r *= n[k];
  return tune_choice(modes12_key(n[0], n[1], r)) != modes12_shape_count();
}

// Tucker chain V x_1 M_1 ... x_d M_d with ping-pong buffers; the last applied
// mode writes through `last` (its out0 and the other fields); earlier modes
// store plainly.  Modes whose matrix is NULL are skipped.  If every matrix is
// NULL the result is V itself, run through an identity mode-1 product is not
// possible, so the caller must not ask for that (checked by tucker_apply).
//
// With a reduced contraction precision the inner modes keep FP32
// intermediates in the ping-pong buffers (half the bytes of FP64) and the
// last mode returns to FP64 through its epilogue.

// Exact-slice chain: per mode, the digits of the current tensor along that
// mode go to dig_ws, and the int8 product writes the FP64 result to t0 (the
// slice kernel has consumed t0 before the product overwrites it).
int tucker_chain_sliced(int d, const int* n, const void* const* M, const void* const* Mdig, const void* V,
                        void* t0, void* dig_ws, const Epilogue& last, void* stream) {
  int lastmu = -1;
  for (int mu = 0; mu < d; ++mu)
    if (M[mu]) lastmu = mu;
  const void* src = V;
  for (int mu = 0; mu < d; ++mu) {
    if (!M[mu]) continue;
    long s, r;
    mode_view(d, n, mu, &s, &r);
    TRY(launch_slice(static_cast<const double*>(src), s, n[mu], r, mu == 0, dig_ws, stream));
    if (mu == lastmu) {
      TRY(launch_sliced_mode_product(s, n[mu], r, mu == 0, Mdig[mu], dig_ws, last, stream));
    } else {
      Epilogue e;
      e.op = EPI_AXPBY;
      e.alpha = 1.0;
      e.beta = 0.0;
      e.out0 = t0;
      TRY(launch_sliced_mode_product(s, n[mu], r, mu == 0, Mdig[mu], dig_ws, e, stream));
      src = t0;
    }
  }
  return EXPINT_OK;
}

int tucker_chain(int dtype, int precision, int d, const int* n, const void* const* M, const void* V,
                 void* t0, void* t1, const Epilogue& last, void* stream, const void* const* Mdig = nullptr,
                 void* dig_ws = nullptr) {
  if (precision == EXPINT_PREC_SLICED) return tucker_chain_sliced(d, n, M, Mdig, V, t0, dig_ws, last, stream);
  int lastmu = -1;
  for (int mu = 0; mu < d; ++mu)
    if (M[mu]) lastmu = mu;
  const bool lp = precision != EXPINT_PREC_FP64;
  const void* src = V;
  bool src32 = false;
  void* bufs[2] = {t0, t1};
  int which = 0;
  // When mode 2 is the last one the fused launch writes the chain's output,
  // which must then not be the input.
  const bool fuse12 = fuse12_allowed(dtype, precision, d, n) && M[0] && M[1] &&
                      (lastmu != 1 || (last.out0 != V && last.out1 != V));
  for (int mu = 0; mu < d; ++mu) {
    if (!M[mu]) continue;
    long s, r;
    if (mu == 0 && fuse12) {
      mode_view(d, n, 1, &s, &r);
      if (lastmu == 1) {
        TRY(launch_modes12(n[0], n[1], r, M[0], M[1], src, last, stream));
      } else {
        Epilogue e;
        e.op = EPI_AXPBY;
        e.alpha = 1.0;
        e.beta = 0.0;
        e.out0 = bufs[which];
        TRY(launch_modes12(n[0], n[1], r, M[0], M[1], src, e, stream));
        src = bufs[which];
        which ^= 1;
      }
      mu = 1;
      continue;
    }
    mode_view(d, n, mu, &s, &r);
    if (mu == lastmu) {
      if (lp)
        TRY(launch_mode_product_lp(precision, dtype == EXPINT_C128, src32, false, s, n[mu], r, M[mu], src, last, stream));
      else
        TRY(launch_mode_product(dtype, s, n[mu], r, M[mu], src, last, stream));
    } else {
      Epilogue e;
      e.op = EPI_AXPBY;
      e.alpha = 1.0;
      e.beta = 0.0;
      e.out0 = bufs[which];
      if (lp)
        TRY(launch_mode_product_lp(precision, dtype == EXPINT_C128, src32, true, s, n[mu], r, M[mu], src, e, stream));
      else
        TRY(launch_mode_product(dtype, s, n[mu], r, M[mu], src, e, stream));
      src = bufs[which];
      src32 = lp;
      which ^= 1;
    }
  }
  return EXPINT_OK;
}



int count_modes(int d, const void* const* M) {
  int c = 0;
  for (int mu = 0; mu < d; ++mu) c += M[mu] != nullptr;
  return c;
}

}  // namespace
}  // namespace expint

using namespace expint;


// ---------------------------------------------------------------------------
// tucker_apply
// ---------------------------------------------------------------------------

extern "C" int tucker_fuses_modes12(int d, const int* n, int dtype, int precision, int* fused) {
  long N;
  TRY(validate_shape(d, n, &N));
  if (dtype != EXPINT_F64 && dtype != EXPINT_C128) return set_error(EXPINT_EINVAL, "unknown dtype %d", dtype);
  if (!valid_precision(precision)) return set_error(EXPINT_EINVAL, "unknown precision %d", precision);
  if (!fused) return set_error(EXPINT_EINVAL, "fused is NULL");
  *fused = fuse12_allowed(dtype, precision, d, n) ? 1 : 0;
  return EXPINT_OK;
}

// Validation shared by tucker_apply and tucker_apply_noalloc: every argument
// except the workspace, then the workspace layout the call needs.
static int tucker_validate(int d, const int* n, const void* const* M, const void* V, void* W, double alpha,
                           double beta, int dtype, int precision, long* N, size_t* tens, size_t* digs,
                           size_t* mdigs) {
  TRY(validate_shape(d, n, N));
  if (dtype != EXPINT_F64 && dtype != EXPINT_C128) return set_error(EXPINT_EINVAL, "unknown dtype %d", dtype);
  if (!valid_precision(precision)) return set_error(EXPINT_EINVAL, "tucker_apply: unknown precision %d", precision);
  if ((precision == EXPINT_PREC_BF16X3 || precision == EXPINT_PREC_SLICED) && dtype != EXPINT_F64)
    return set_error(EXPINT_ENOTSUP, "tucker_apply: complex data supports FP64 or FP32 (complex64) contraction");
  TRY(check_operand_limits(d, n, *N, dtype, precision));
  if (!M || !V || !W) return set_error(EXPINT_EINVAL, "tucker_apply: NULL M, V or W");
  if (V == W) return set_error(EXPINT_EINVAL, "tucker_apply: V must not alias W");
  if (!aligned16(V) || !aligned16(W)) return set_error(EXPINT_EINVAL, "tucker_apply: V and W must be 16-byte aligned");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return set_error(EXPINT_EINVAL, "tucker_apply: alpha/beta not finite");
  for (int mu = 0; mu < d; ++mu)
    if (M[mu] && !aligned16(M[mu])) return set_error(EXPINT_EINVAL, "tucker_apply: M[%d] not 16-byte aligned", mu);
  const int modes = count_modes(d, M);
  if (modes == 0) return set_error(EXPINT_EINVAL, "tucker_apply: every M[mu] is NULL (nothing to apply)");
  return tucker_ws_layout(d, n, *N, dtype, precision, modes, tens, digs, mdigs);
}

// The kernel sequence of a validated Tucker operator, with its workspace at w.
static int tucker_enqueue(int d, const int* n, const void* const* M, const void* V, void* W, double alpha,
                          double beta, int dtype, int precision, long N, size_t tens, size_t digs, char* w,
                          void* stream) {
  Epilogue last;
  last.op = EPI_AXPBY;
  last.alpha = alpha;
  last.beta = beta;
  last.out0 = W;
  if (precision == EXPINT_PREC_SLICED) {
    // digits of each M (rows along its columns), then the chain
    const void* Md[4] = {nullptr, nullptr, nullptr, nullptr};
    char* mp = w + tens + digs;
    for (int mu = 0; mu < d; ++mu) {
      if (!M[mu]) continue;
      TRY(launch_slice(static_cast<const double*>(M[mu]), n[mu], n[mu], 1, false, mp, stream));
      Md[mu] = mp;
      mp += slice_digits_bytes(n[mu], n[mu]);
    }
    return tucker_chain(dtype, precision, d, n, M, V, tens ? w : nullptr, nullptr, last, stream, Md, w + tens);
  }
  void* t0 = tens ? w : nullptr;
  void* t1 = tens ? w + (size_t)N * elem_size(dtype) : nullptr;
  return tucker_chain(dtype, precision, d, n, M, V, t0, t1, last, stream);
}

extern "C" int tucker_apply(int d, const int* n, const void* const* M, const void* V, void* W,
                            double alpha, double beta, int dtype, int precision, void* ws,
                            size_t ws_bytes, void* stream) {
  long N;
  size_t tens, digs, mdigs;
  TRY(tucker_validate(d, n, M, V, W, alpha, beta, dtype, precision, &N, &tens, &digs, &mdigs));
  const size_t need = tens + digs + mdigs;
  if (ws_bytes < need || (need > 0 && !ws))
    return set_error(EXPINT_EINVAL, "tucker_apply: workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (need > 0 && !aligned16(ws)) return set_error(EXPINT_EINVAL, "tucker_apply: workspace not 16-byte aligned");
  return tucker_enqueue(d, n, M, V, W, alpha, beta, dtype, precision, N, tens, digs, static_cast<char*>(ws),
                        stream);
}

// ---------------------------------------------------------------------------
// tucker_apply_noalloc: the same kernels with the workspace in a fixed device array
// ---------------------------------------------------------------------------

// The intermediates of tucker_apply_noalloc.  Each device holds its own copy
// for the life of the process; host code never passes this name to a kernel
// or a copy (on the host it is a stand-in, not a device address) but the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[EXPINT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return set_error(EXPINT_ENOTSUP, "tucker_apply_noalloc: device ordinal %d beyond %d", dev, kScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(EXPINT_EHIP, "tucker_apply_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return EXPINT_OK;
}
}  // namespace

extern "C" int tucker_apply_noalloc(int d, const int* n, const void* const* M, const void* V, void* W,
                                    double alpha, double beta, int dtype, int precision, void* stream) {
  long N;
  size_t tens, digs, mdigs;
  TRY(tucker_validate(d, n, M, V, W, alpha, beta, dtype, precision, &N, &tens, &digs, &mdigs));
  const size_t need = tens + digs + mdigs;
  if (need > (size_t)EXPINT_NOALLOC_SCRATCH_BYTES)
    return set_error(EXPINT_ENOTSUP,
                     "tucker_apply_noalloc: this shape needs %zu bytes of scratch, the fixed limit is %zu bytes "
                     "(use tucker_apply with a workspace)",
                     need, (size_t)EXPINT_NOALLOC_SCRATCH_BYTES);
  void* ptr = nullptr;
  if (need > 0) TRY(scratch_address(&ptr));
  return tucker_enqueue(d, n, M, V, W, alpha, beta, dtype, precision, N, tens, digs, static_cast<char*>(ptr),
                        stream);
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

struct expint_plan {
  int d = 0;
  int n[4] = {1, 1, 1, 1};
  long N = 0;
  double tau = 0.0;
  int scheme = 0, nonlin = 0, dtype = 0, precision = 0;
  double gparam = 0.0;
  int ell_lo = 0, ell_hi = 0;        // phi indices the scheme uses
  void* phi[4][3] = {};              // device phi_l(tau A_mu); shared between equal directions
  bool phi_owner[4][3] = {};
  void* phidig[4][3] = {};           // exact-slice digits of phi (EXPINT_PREC_SLICED); always owned
  bool use_stencil = false;
  Stencil stencil;                   // device coefficient arrays when use_stencil
  void* denseA[4] = {};              // device A_mu for the dense K u path
  int device = 0;
  // coordinate / time dependent nonlinearity
  GridTime gt;
  double* d_clock = nullptr;
  bool timedep = false;
  bool small = false;                // whole runs in one fused launch (small 2-D FP64 problems)
  int* d_flag = nullptr;             // device int of expint_plan_check_finite
  // cached graph of one step
  hipGraphExec_t gexec = nullptr;
  const void* g_U = nullptr;
  const void* g_ws = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace {

int classify_tridiagonal(int n, const double* A, int cplx, bool* tri, bool* periodic) {
  const int w = cplx ? 2 : 1;
  auto nz = [&](int i, int j) {
    const double* p = A + ((size_t)i + (size_t)n * j) * w;
    return p[0] != 0.0 || (cplx && p[1] != 0.0);
  };
  *tri = true;
  *periodic = false;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const int dist = i > j ? i - j : j - i;
      if (dist <= 1 || !nz(i, j)) continue;
      if (n >= 3 && ((i == 0 && j == n - 1) || (i == n - 1 && j == 0))) {
        *periodic = true;
        continue;
      }
      *tri = false;
      return EXPINT_OK;
    }
  return EXPINT_OK;
}

void free_plan_memory(expint_plan* p) {
  for (int mu = 0; mu < 4; ++mu) {
    for (int l = 0; l < 3; ++l)
      if (p->phi_owner[mu][l] && p->phi[mu][l]) (void)hipFree(p->phi[mu][l]);
    for (int l = 0; l < 3; ++l)
      if (p->phidig[mu][l]) (void)hipFree(p->phidig[mu][l]);
    if (p->stencil.coef[mu]) (void)hipFree(const_cast<void*>(p->stencil.coef[mu]));
    if (p->denseA[mu]) (void)hipFree(p->denseA[mu]);
  }
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->d_clock) (void)hipFree(p->d_clock);
  if (p->d_flag) (void)hipFree(p->d_flag);
}

int scheme_phi_range(int scheme, int* lo, int* hi) {
  switch (scheme) {
    case EXPINT_LAWSON_EULER:
    case EXPINT_LAWSON2B:
      *lo = 0;
      *hi = 0;
      return EXPINT_OK;
    case EXPINT_EXP_EULER:
      *lo = 1;
      *hi = 1;
      return EXPINT_OK;
    case EXPINT_ETD2RK:
      *lo = 1;
      *hi = 2;
      return EXPINT_OK;
    default:
      return set_error(EXPINT_EINVAL, "unknown scheme %d", scheme);
  }
}

int workspace_elems(const expint_plan* p, long* elems) {
  // buffers: W (stage input), T0, T1 (Tucker ping-pong), X (U_n2 / W_b), Y (Lawson2b U_n2)
  long k = 0;
  switch (p->scheme) {
    case EXPINT_LAWSON_EULER:
    case EXPINT_EXP_EULER:
      k = 3;
      break;
    case EXPINT_ETD2RK:
      k = 4;
      break;
    case EXPINT_LAWSON2B:
      k = 5;
      break;
  }
  *elems = k * p->N;
  return EXPINT_OK;
}

// extra bytes after the scheme's tensors: the digit buffer of the exact-slice chain
size_t workspace_extra_bytes(const expint_plan* p) {
  if (p->precision != EXPINT_PREC_SLICED) return 0;
  return 256 + sliced_tensor_digits_bytes(p->d, p->n, p->N);  // 256: room to align the digit buffer
}

// digits of phi_ell(tau A_mu) for the exact-slice contraction (synchronous)
int slice_phi(expint_plan* p, int mu, int ell) {
  const int n = p->n[mu];
  if (!p->phidig[mu][ell]) {
    void* dptr = nullptr;
    if (hipMalloc(&dptr, slice_digits_bytes(n, n)) != hipSuccess)
      return set_error(EXPINT_ENOMEM, "device allocation for phi digits failed");
    p->phidig[mu][ell] = dptr;
  }
  TRY(launch_slice(static_cast<const double*>(p->phi[mu][ell]), n, n, 1, false, p->phidig[mu][ell], nullptr));
  HIP_TRY(hipStreamSynchronize(nullptr));
  return EXPINT_OK;
}

// stage input W = tau (K U + g(U))
int stage_input(expint_plan* p, const void* U, void* W, hipStream_t s) {
  if (p->use_stencil)
    return launch_stage_stencil(p->dtype, p->stencil, p->N, U, W, p->tau, p->nonlin, p->gparam, p->gt, s);
  TRY(launch_scaled_g(p->dtype, p->N, U, W, p->tau, p->nonlin, p->gparam, p->gt, s));
  for (int mu = 0; mu < p->d; ++mu) {
    long sv, rv;
    mode_view(p->d, p->n, mu, &sv, &rv);
    Epilogue e;
    e.op = EPI_AXPBY;
    e.alpha = p->tau;
    e.beta = 1.0;
    e.out0 = W;
    TRY(launch_mode_product(p->dtype, sv, p->n[mu], rv, p->denseA[mu], U, e, s));
  }
  return EXPINT_OK;
}

int enqueue_step_body(expint_plan* p, void* U, void* ws, hipStream_t s);

// one step; a time-dependent g also advances the device clock at the end
int enqueue_step(expint_plan* p, void* U, void* ws, hipStream_t s) {
  TRY(enqueue_step_body(p, U, ws, s));
  if (p->timedep) TRY(launch_clock_tick(p->d_clock, s));
  return EXPINT_OK;
}

int enqueue_step_body(expint_plan* p, void* U, void* ws, hipStream_t s) {
  const size_t es = elem_size(p->dtype);
  char* base = static_cast<char*>(ws);
  void* W = base;
  void* T0 = base + 1 * p->N * es;
  void* T1 = base + 2 * p->N * es;
  void* X = base + 3 * p->N * es;
  void* Y = base + 4 * p->N * es;
  const void* P0[4] = {p->phi[0][0], p->phi[1][0], p->phi[2][0], p->phi[3][0]};
  const void* P1[4] = {p->phi[0][1], p->phi[1][1], p->phi[2][1], p->phi[3][1]};
  const void* P2[4] = {p->phi[0][2], p->phi[1][2], p->phi[2][2], p->phi[3][2]};
  const void* D0[4] = {p->phidig[0][0], p->phidig[1][0], p->phidig[2][0], p->phidig[3][0]};
  const void* D1[4] = {p->phidig[0][1], p->phidig[1][1], p->phidig[2][1], p->phidig[3][1]};
  const void* D2[4] = {p->phidig[0][2], p->phidig[1][2], p->phidig[2][2], p->phidig[3][2]};
  long elems;
  TRY(workspace_elems(p, &elems));
  // exact-slice digit buffer, 256-byte aligned after the scheme's tensors
  void* DG = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(base + (size_t)elems * es) + 255) & ~uintptr_t(255));
  const double split2 = std::ldexp(1.0, p->d - 1);  // (2!)^{d-1}
  switch (p->scheme) {
    case EXPINT_LAWSON_EULER: {
      // U_{n+1} = (U_n + tau G_n) x_mu e^{tau A_mu}
      TRY(launch_lawson_stage(p->dtype, p->N, U, W, nullptr, p->tau, p->nonlin, p->gparam, p->gt, s));
      Epilogue e;
      e.op = EPI_AXPBY;
      e.out0 = U;
      return tucker_chain(p->dtype, p->precision, p->d, p->n, P0, W, T0, T1, e, s, D0, DG);
    }
    case EXPINT_LAWSON2B: {
      // U_n2 = (U_n + tau G_n) x e^{tau A};  U_{n+1} = (U_n + tau/2 G_n) x e^{tau A} + tau/2 G(U_n2)
      TRY(launch_lawson_stage(p->dtype, p->N, U, W, X, p->tau, p->nonlin, p->gparam, p->gt, s));
      Epilogue e1;
      e1.op = EPI_AXPBY;
      e1.out0 = Y;
      TRY(tucker_chain(p->dtype, p->precision, p->d, p->n, P0, W, T0, T1, e1, s, D0, DG));
      Epilogue e2;
      e2.op = EPI_LAWSON2B_2;
      e2.out0 = U;
      e2.in1 = Y;
      e2.c = 0.5 * p->tau;
      e2.g = p->nonlin;
      e2.gparam = p->gparam;
      e2.gt = p->gt;
      return tucker_chain(p->dtype, p->precision, p->d, p->n, P0, X, T0, T1, e2, s, D0, DG);
    }
    case EXPINT_EXP_EULER: {
      // U_{n+1} = U_n + (tau (K U_n + G_n)) x_mu phi_1(tau A_mu)   ((1!)^{d-1} = 1)
      TRY(stage_input(p, U, W, s));
      Epilogue e;
      e.op = EPI_EXP_EULER;
      e.out0 = U;
      e.in1 = U;
      return tucker_chain(p->dtype, p->precision, p->d, p->n, P1, W, T0, T1, e, s, D1, DG);
    }
    case EXPINT_ETD2RK: {
      // U_n2 = U_n + (tau (K U_n + G_n)) x phi_1;  W_2 = tau (G(U_n2) - G_n)
      // U_{n+1} = U_n2 + (2!)^{d-1} W_2 x phi_2
      TRY(stage_input(p, U, W, s));
      Epilogue e1;
      e1.op = EPI_ETD2RK_1;
      e1.out0 = X;  // U_n2
      e1.in1 = U;
      e1.out1 = W;  // W_2 (the first stage input is no longer needed once mode 1 has read it)
      e1.tau = p->tau;
      e1.g = p->nonlin;
      e1.gparam = p->gparam;
      e1.gt = p->gt;
      if (count_modes(p->d, P1) == 1) {
        // a single mode reads W while its epilogue writes W_2: keep them apart
        e1.out1 = T1;
        TRY(tucker_chain(p->dtype, p->precision, p->d, p->n, P1, W, T0, nullptr, e1, s, D1, DG));
        W = T1;
      } else {
        TRY(tucker_chain(p->dtype, p->precision, p->d, p->n, P1, W, T0, T1, e1, s, D1, DG));
      }
      Epilogue e2;
      e2.op = EPI_ETD2RK_2;
      e2.out0 = U;
      e2.in1 = X;
      e2.c = split2;
      return tucker_chain(p->dtype, p->precision, p->d, p->n, P2, W, T0, T1, e2, s, D2, DG);
    }
  }
  return set_error(EXPINT_EINVAL, "unknown scheme");
}

int validate_step_args(expint_plan* p, void* U, void* ws) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  if (!U || !ws) return set_error(EXPINT_EINVAL, "U and ws must be non-NULL device pointers");
  if (!aligned16(U) || !aligned16(ws)) return set_error(EXPINT_EINVAL, "U and ws must be 16-byte aligned");
  return EXPINT_OK;
}

}  // namespace

extern "C" int expint_plan_create(expint_plan** out, const expint_problem* prob) {
  if (!out) return set_error(EXPINT_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  if (!prob) return set_error(EXPINT_EINVAL, "problem is NULL");
  if (prob->d < 1 || prob->d > 4) return set_error(EXPINT_EINVAL, "d = %d: need 1 <= d <= 4", prob->d);
  long N;
  TRY(validate_shape(prob->d, prob->n, &N));
  if (prob->dtype != EXPINT_F64 && prob->dtype != EXPINT_C128)
    return set_error(EXPINT_EINVAL, "unknown dtype %d", prob->dtype);
  if (!valid_precision(prob->precision)) return set_error(EXPINT_EINVAL, "unknown precision %d", prob->precision);
  if (prob->phi_method != EXPINT_PHI_TAYLOR && prob->phi_method != EXPINT_PHI_QUAD)
    return set_error(EXPINT_EINVAL, "unknown phi construction %d", prob->phi_method);
  if ((prob->precision == EXPINT_PREC_BF16X3 || prob->precision == EXPINT_PREC_SLICED) && prob->dtype != EXPINT_F64)
    return set_error(EXPINT_ENOTSUP, "complex data supports FP64 or FP32 (complex64) contraction");
  if (!std::isfinite(prob->tau)) return set_error(EXPINT_EINVAL, "tau is not finite");
  TRY(check_operand_limits(prob->d, prob->n, N, prob->dtype, prob->precision));
  const bool cplx = prob->dtype == EXPINT_C128;
  if (cplx && prob->nonlin != EXPINT_G_NONE && prob->nonlin != EXPINT_G_CUBIC_NLS)
    return set_error(EXPINT_ENOTSUP, "complex data supports g = NONE or CUBIC_NLS");
  if (!cplx && prob->nonlin != EXPINT_G_NONE && prob->nonlin != EXPINT_G_ALLEN_CAHN &&
      prob->nonlin != EXPINT_G_U2_1MU && prob->nonlin != EXPINT_G_ADR_PAPER)
    return set_error(EXPINT_ENOTSUP, "real data supports g = NONE, ALLEN_CAHN, U2_1MU or ADR_PAPER");
  if (prob->nonlin == EXPINT_G_ADR_PAPER && prob->d != 3)
    return set_error(EXPINT_ENOTSUP, "EXPINT_G_ADR_PAPER is defined for d = 3");
  int lo, hi;
  TRY(scheme_phi_range(prob->scheme, &lo, &hi));
  for (int mu = 0; mu < prob->d; ++mu)
    if (!prob->A[mu]) return set_error(EXPINT_EINVAL, "A[%d] is NULL", mu);

  expint_plan* p = new (std::nothrow) expint_plan();
  if (!p) return set_error(EXPINT_ENOMEM, "plan allocation failed");
  p->d = prob->d;
  for (int mu = 0; mu < prob->d; ++mu) p->n[mu] = prob->n[mu];
  p->N = N;
  p->tau = prob->tau;
  p->scheme = prob->scheme;
  p->nonlin = prob->nonlin;
  p->gparam = prob->g_param;
  p->timedep = prob->nonlin == EXPINT_G_ADR_PAPER;
  for (int mu = 0; mu < 3 && mu < prob->d; ++mu) {
    p->gt.n[mu] = prob->n[mu];
    p->gt.h[mu] = 1.0 / (prob->n[mu] + 1);
  }
  p->gt.eps = prob->g_param;
  p->gt.alpha = prob->g_param2;
  p->gt.tau = prob->tau;
  p->dtype = prob->dtype;
  p->precision = prob->precision;
  p->ell_lo = lo;
  p->ell_hi = hi;
  (void)hipGetDevice(&p->device);
  const size_t es = elem_size(p->dtype);
  int rc = EXPINT_OK;

  // phi matrices: built once per distinct A_mu (section 3.1 / 4.2)
  for (int mu = 0; mu < p->d && rc == EXPINT_OK; ++mu) {
    const int n = p->n[mu];
    const size_t bytes = (size_t)n * n * es;
    int same = -1;
    for (int nu = 0; nu < mu; ++nu)
      if (p->n[nu] == n && std::memcmp(prob->A[nu], prob->A[mu], bytes) == 0) same = nu;
    if (same >= 0) {
      for (int l = lo; l <= hi; ++l) p->phi[mu][l] = p->phi[same][l];
      continue;
    }
    std::vector<double> host;
    try {
      host.resize((size_t)(hi + 1) * n * n * (cplx ? 2 : 1));
    } catch (const std::bad_alloc&) {
      rc = set_error(EXPINT_ENOMEM, "host allocation for phi failed");
      break;
    }
    rc = phi_setup_method(prob->phi_method, cplx, n, prob->A[mu], n, p->tau, hi, host.data(), n);
    for (int l = lo; l <= hi && rc == EXPINT_OK; ++l) {
      void* dptr = nullptr;
      if (hipMalloc(&dptr, bytes) != hipSuccess) {
        rc = set_error(EXPINT_ENOMEM, "device allocation for phi failed");
        break;
      }
      p->phi[mu][l] = dptr;
      p->phi_owner[mu][l] = true;
      if (hipMemcpy(dptr, host.data() + (size_t)l * n * n * (cplx ? 2 : 1), bytes, hipMemcpyHostToDevice) !=
          hipSuccess)
        rc = set_error(EXPINT_EHIP, "copy of phi to the device failed");
    }
  }

  // exact-slice digits of every phi the scheme uses
  if (rc == EXPINT_OK && p->precision == EXPINT_PREC_SLICED)
    for (int mu = 0; mu < p->d && rc == EXPINT_OK; ++mu)
      for (int l = lo; l <= hi && rc == EXPINT_OK; ++l) rc = slice_phi(p, mu, l);

  // operator data for K u: stencil if every A_mu is (periodic) tridiagonal, else dense
  if (rc == EXPINT_OK && (p->scheme == EXPINT_EXP_EULER || p->scheme == EXPINT_ETD2RK)) {
    bool all_tri = true;
    bool per[4] = {false, false, false, false};
    for (int mu = 0; mu < p->d; ++mu) {
      bool tri, periodic;
      classify_tridiagonal(p->n[mu], prob->A[mu], cplx, &tri, &periodic);
      all_tri = all_tri && tri;
      per[mu] = periodic;
    }
    p->use_stencil = all_tri;
    p->stencil.d = p->d;
    bool all_toeplitz = true;
    for (int mu = 0; mu < p->d && rc == EXPINT_OK; ++mu) {
      const int n = p->n[mu];
      const int w = cplx ? 2 : 1;
      const double* A = prob->A[mu];
      if (all_tri) {
        std::vector<double> c;
        try {
          c.assign((size_t)3 * n * w, 0.0);
        } catch (const std::bad_alloc&) {
          rc = set_error(EXPINT_ENOMEM, "host allocation for the stencil failed");
          break;
        }
        auto put = [&](int slot, int i, int row, int col) {
          for (int k = 0; k < w; ++k) c[((size_t)slot * n + i) * w + k] = A[((size_t)row + (size_t)n * col) * w + k];
        };
        for (int i = 0; i < n; ++i) {
          put(1, i, i, i);
          if (i > 0) put(0, i, i, i - 1);
          if (i < n - 1) put(2, i, i, i + 1);
        }
        if (per[mu]) {
          put(0, 0, 0, n - 1);
          put(2, n - 1, n - 1, 0);
        }
        // Toeplitz: the entries that are used are constant along each diagonal
        bool toep = true;
        for (int slot = 0; slot < 3 && toep; ++slot)
          for (int i = 0; i < n && toep; ++i) {
            if ((slot == 0 && i == 0 && !per[mu]) || (slot == 2 && i == n - 1 && !per[mu])) continue;
            const int ref = (slot == 0 && !per[mu]) ? 1 : 0;
            for (int k = 0; k < w; ++k)
              if (c[((size_t)slot * n + i) * w + k] != c[((size_t)slot * n + ref) * w + k]) toep = false;
          }
        all_toeplitz = all_toeplitz && toep;
        for (int slot = 0; slot < 3; ++slot) {
          const int ref = (slot == 0 && !per[mu] && n > 1) ? 1 : 0;
          for (int k = 0; k < w; ++k) p->stencil.tc[mu][slot][k] = c[((size_t)slot * n + ref) * w + k];
        }
        void* dptr = nullptr;
        if (hipMalloc(&dptr, c.size() * sizeof(double)) != hipSuccess) {
          rc = set_error(EXPINT_ENOMEM, "device allocation for stencil failed");
          break;
        }
        p->stencil.coef[mu] = dptr;
        p->stencil.n[mu] = n;
        p->stencil.periodic[mu] = per[mu] ? 1 : 0;
        if (hipMemcpy(dptr, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
          rc = set_error(EXPINT_EHIP, "copy of stencil to the device failed");
        p->stencil.toeplitz = all_toeplitz;
      } else {
        const size_t bytes = (size_t)n * n * es;
        void* dptr = nullptr;
        if (hipMalloc(&dptr, bytes) != hipSuccess) {
          rc = set_error(EXPINT_ENOMEM, "device allocation for A failed");
          break;
        }
        p->denseA[mu] = dptr;
        if (hipMemcpy(dptr, A, bytes, hipMemcpyHostToDevice) != hipSuccess)
          rc = set_error(EXPINT_EHIP, "copy of A to the device failed");
      }
    }
  }
  if (rc == EXPINT_OK && p->timedep) {
    if (hipMalloc(&p->d_clock, 2 * sizeof(double)) != hipSuccess) {
      rc = set_error(EXPINT_ENOMEM, "device allocation for the clock failed");
    } else {
      const double zero[2] = {0.0, 0.0};
      if (hipMemcpy(p->d_clock, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
        rc = set_error(EXPINT_EHIP, "clock initialisation failed");
      p->gt.clock = p->d_clock;
    }
  }
  if (rc == EXPINT_OK) {
    if (hipMalloc(&p->d_flag, sizeof(int)) != hipSuccess)
      rc = set_error(EXPINT_ENOMEM, "device allocation for the status flag failed");
    else if (hipMemset(p->d_flag, 0, sizeof(int)) != hipSuccess)
      rc = set_error(EXPINT_EHIP, "status flag initialisation failed");
  }
  if (rc != EXPINT_OK) {
    free_plan_memory(p);
    delete p;
    return rc;
  }
  {
    const char* env = std::getenv("EXPINT_SMALL_FUSED");
    const bool allowed = !(env && env[0] == '0');
    p->small = allowed && small2d_fits(p->d, p->n) && p->dtype == EXPINT_F64 &&
               p->precision == EXPINT_PREC_FP64 && !p->timedep;
  }
  if (prob->tune && !p->small) {
    const int trc = tune_tucker_shapes(p->d, p->n, p->dtype, p->precision, nullptr);
    if (trc != EXPINT_OK) {
      free_plan_memory(p);
      delete p;
      return trc;
    }
  }
  *out = p;
  return EXPINT_OK;
}

extern "C" int expint_plan_describe(const expint_plan* p, char* buf, size_t len, size_t* needed) {
  if (!p || (!buf && len > 0)) return set_error(EXPINT_EINVAL, "NULL plan or buffer");
  std::string s;
  if (p->small) {
    s = "k_small2d: whole run in one workgroup\n";
  } else if (p->precision == EXPINT_PREC_FP64 || p->precision == EXPINT_PREC_SLICED) {
    const bool f12 = fuse12_allowed(p->dtype, p->precision, p->d, p->n);
    if (p->precision == EXPINT_PREC_FP64 && p->dtype == EXPINT_F64 && p->d >= 2 && modes12_fits(p->n[0], p->n[1])) {
      long r = 1;
      for (int k = 2; k < p->d; ++k) r *= p->n[k];
      s += tune_describe(modes12_key(p->n[0], p->n[1], r)) + (f12 ? " [fused]\n" : " [not fused]\n");
    }
    for (int mu = 0; mu < p->d; ++mu) {
      long sv, rv;
      mode_view(p->d, p->n, mu, &sv, &rv);
      const TuneKey k = p->precision == EXPINT_PREC_SLICED ? sliced_key(sv, p->n[mu], rv)
                                                            : mode_product_key(p->dtype == EXPINT_C128, sv, p->n[mu], rv);
      s += "mode " + std::to_string(mu + 1) + ": " + tune_describe(k) + "\n";
    }
  } else if (p->dtype == EXPINT_F64) {
    for (int mu = 0; mu < p->d; ++mu) {
      long sv, rv;
      mode_view(p->d, p->n, mu, &sv, &rv);
      s += "mode " + std::to_string(mu + 1) + ": " + tune_describe(lp_key(p->precision, sv, p->n[mu], rv)) + "\n";
    }
  } else {
    s = "complex64 mu-mode products: one configuration\n";
  }
  if (needed) *needed = s.size() + 1;
  if (len > 0) {
    const size_t m = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), m);
    buf[m] = '\0';
  }
  return EXPINT_OK;
}

extern "C" int expint_plan_workspace_size(const expint_plan* p, size_t* bytes) {
  if (!p || !bytes) return set_error(EXPINT_EINVAL, "NULL plan or output");
  long elems;
  TRY(workspace_elems(p, &elems));
  *bytes = (size_t)elems * elem_size(p->dtype) + workspace_extra_bytes(p);
  return EXPINT_OK;
}

extern "C" int expint_plan_set_phi(expint_plan* p, int mu, int ell, const double* host_phi) {
  if (!p || !host_phi) return set_error(EXPINT_EINVAL, "NULL plan or matrix");
  if (mu < 0 || mu >= p->d) return set_error(EXPINT_EINVAL, "direction %d out of range", mu);
  if (ell < p->ell_lo || ell > p->ell_hi)
    return set_error(EXPINT_EINVAL, "phi_%d is not used by this scheme", ell);
  const int n = p->n[mu];
  const size_t bytes = (size_t)n * n * elem_size(p->dtype);
  // Directions with equal A share one device matrix.  Only direction mu
  // changes: if any other direction still points at mu's matrix, mu moves to
  // a fresh allocation (an owner hands its old matrix to the first sharer), so
  // the sharers keep the matrix, and the digits, they had.
  bool shared = false;
  for (int nu = 0; nu < p->d; ++nu)
    if (nu != mu && p->phi[nu][ell] == p->phi[mu][ell]) shared = true;
  if (shared) {
    void* dptr = nullptr;
    if (hipMalloc(&dptr, bytes) != hipSuccess) return set_error(EXPINT_ENOMEM, "device allocation failed");
    void* old = p->phi[mu][ell];
    if (p->phi_owner[mu][ell]) {
      for (int nu = 0; nu < p->d; ++nu)
        if (nu != mu && p->phi[nu][ell] == old) {
          p->phi_owner[nu][ell] = true;
          break;
        }
    }
    p->phi[mu][ell] = dptr;
    p->phi_owner[mu][ell] = true;
    if (p->gexec) {  // the captured step holds the old pointer
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
  }
  HIP_TRY(hipMemcpy(p->phi[mu][ell], host_phi, bytes, hipMemcpyHostToDevice));
  if (p->precision == EXPINT_PREC_SLICED) TRY(slice_phi(p, mu, ell));
  return EXPINT_OK;
}

extern "C" int expint_plan_is_fused(const expint_plan* p, int* fused) {
  if (!p || !fused) return set_error(EXPINT_EINVAL, "NULL plan or output");
  *fused = p->small ? 1 : 0;
  return EXPINT_OK;
}

// all steps of a small 2-D problem in one fused launch
static int run_small(expint_plan* p, void* U, int nsteps, void* stream) {
  SmallArgs a;
  a.U = static_cast<double*>(U);
  for (int mu = 0; mu < 2; ++mu) {
    for (int l = 0; l < 3; ++l) a.M[mu][l] = static_cast<const double*>(p->phi[mu][l]);
    a.stc[mu] = static_cast<const double*>(p->stencil.coef[mu]);
    a.periodic[mu] = p->stencil.periodic[mu];
    a.A[mu] = static_cast<const double*>(p->denseA[mu]);
  }
  a.stencil = p->use_stencil ? 1 : 0;
  a.n1 = p->n[0];
  a.n2 = p->n[1];
  a.tau = p->tau;
  a.gparam = p->gparam;
  a.scheme = p->scheme;
  a.g = p->nonlin;
  a.nsteps = nsteps;
  return launch_small2d(a, stream);
}

extern "C" int expint_step(expint_plan* p, void* U, double t, void* ws, void* stream) {
  TRY(validate_step_args(p, U, ws));
  if (!std::isfinite(t)) return set_error(EXPINT_EINVAL, "t is not finite");
  if (p->small) return run_small(p, U, 1, stream);
  if (p->timedep) TRY(launch_clock_set(p->d_clock, t, stream));
  return enqueue_step(p, U, ws, static_cast<hipStream_t>(stream));
}

extern "C" int expint_run(expint_plan* p, void* U, double t0, int nsteps, int use_graph, void* ws,
                          void* stream) {
  TRY(validate_step_args(p, U, ws));
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps < 0");
  if (!std::isfinite(t0)) return set_error(EXPINT_EINVAL, "t0 is not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->small) return run_small(p, U, nsteps, stream);
  // t_n = t0 + n tau for the steps below (the captured step advances n)
  if (p->timedep) TRY(launch_clock_set(p->d_clock, t0, s));
  if (!use_graph) {
    for (int k = 0; k < nsteps; ++k) TRY(enqueue_step(p, U, ws, s));
    return EXPINT_OK;
  }
  if (!s) return set_error(EXPINT_EINVAL, "graph capture needs a non-default stream");
  if (!(p->gexec && p->g_U == U && p->g_ws == ws && p->g_stream == s)) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_step(p, U, ws, s);
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != EXPINT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) return set_error(EXPINT_EHIP, "stream capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      p->gexec = nullptr;
      return set_error(EXPINT_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    p->g_U = U;
    p->g_ws = ws;
    p->g_stream = s;
  }
  for (int k = 0; k < nsteps; ++k) HIP_TRY(hipGraphLaunch(p->gexec, s));
  return EXPINT_OK;
}

extern "C" int expint_plan_check_finite(expint_plan* p, const void* U, void* stream) {
  if (!p || !U) return set_error(EXPINT_EINVAL, "NULL plan or state");
  if (!aligned16(U)) return set_error(EXPINT_EINVAL, "U must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long count = p->N * (p->dtype == EXPINT_C128 ? 2 : 1);
  TRY(launch_finite_check(static_cast<const double*>(U), count, p->d_flag, s));
  int flag = 0;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    HIP_TRY(hipMemset(p->d_flag, 0, sizeof(int)));
    HIP_TRY(hipDeviceSynchronize());
    return set_error(EXPINT_ENONFINITE, "the state holds inf or nan");
  }
  return EXPINT_OK;
}

extern "C" void expint_plan_destroy(expint_plan* p) {
  if (!p) return;
  free_plan_memory(p);
  delete p;
}


