// Stage-input kernels: the K u action by a 3-point stencil per direction and
// the pointwise nonlinearity g (paper section 3.2: K u_n is applied in tensor
// form as sum_mu U x_mu A_mu, without assembling K).  These kernels are
// bound by HBM traffic: each reads U once (neighbours come from cache) and
// writes its outputs once.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace expint {
namespace {

constexpr int kThreads = 256;

struct StencilArgs {
  long N;
  int d;
  int n[4];
  int periodic[4];
  const void* coef[4];
  const void* U;
  void* W;
  double tau;
  int g;
  double gparam;
};

// One thread per element.  N < 2^31, so 32-bit index arithmetic is exact; the
// direction count D is a template parameter so the direction loop unrolls.
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void k_stage_stencil(StencilArgs a) {
  const unsigned e = blockIdx.x * (unsigned)kThreads + threadIdx.x;
  if (e >= (unsigned)a.N) return;
  const T* U = static_cast<const T*>(a.U);
  const T u = U[e];
  T acc = zero<T>();
  unsigned rem = e, stride = 1;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    const unsigned nm = (unsigned)a.n[mu];
    unsigned i;
    if (mu < D - 1) {
      i = rem % nm;
      rem /= nm;
    } else {
      i = rem;
    }
    const T* c = static_cast<const T*>(a.coef[mu]);
    acc = fma_t(c[nm + i], u, acc);
    if (i > 0)
      acc = fma_t(c[i], U[e - stride], acc);
    else if (a.periodic[mu])
      acc = fma_t(c[i], U[e + (nm - 1) * stride], acc);
    if (i + 1 < nm)
      acc = fma_t(c[2 * nm + i], U[e + stride], acc);
    else if (a.periodic[mu])
      acc = fma_t(c[2 * nm + i], U[e - (nm - 1) * stride], acc);
    stride *= nm;
  }
  static_cast<T*>(a.W)[e] = scale(add(acc, g_eval(a.g, u, a.gparam)), a.tau);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scaled_g(long N, const void* Uv, void* Wv, double s,
                                                       int g, double gp) {
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  if (e >= N) return;
  static_cast<T*>(Wv)[e] = scale(g_eval(g, static_cast<const T*>(Uv)[e], gp), s);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_lawson_stage(long N, const void* Uv, void* Wa, void* Wb,
                                                           double tau, int g, double gp) {
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  if (e >= N) return;
  const T u = static_cast<const T*>(Uv)[e];
  const T gu = g_eval(g, u, gp);
  static_cast<T*>(Wa)[e] = add(u, scale(gu, tau));
  if (Wb) static_cast<T*>(Wb)[e] = add(u, scale(gu, 0.5 * tau));
}

inline unsigned blocks_for(long N) { return (unsigned)((N + kThreads - 1) / kThreads); }

int check_launch(const char* what) {
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "%s: launch failed: %s", what, hipGetErrorString(err));
  return EXPINT_OK;
}

}  // namespace

int launch_stage_stencil(int dtype, const Stencil& st, long N, const void* U, void* W, double tau,
                         int g, double gparam, void* stream) {
  if (N <= 0) return EXPINT_OK;
  StencilArgs a;
  a.N = N;
  a.d = st.d;
  for (int mu = 0; mu < 4; ++mu) {
    a.n[mu] = st.n[mu];
    a.periodic[mu] = st.periodic[mu];
    a.coef[mu] = st.coef[mu];
  }
  a.U = U;
  a.W = W;
  a.tau = tau;
  a.g = g;
  a.gparam = gparam;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(blocks_for(N)), block(kThreads);
  const bool c = dtype == EXPINT_C128;
  switch (st.d) {
    case 1:
      if (c) hipLaunchKernelGGL((k_stage_stencil<cdouble, 1>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_stage_stencil<double, 1>), grid, block, 0, s, a);
      break;
    case 2:
      if (c) hipLaunchKernelGGL((k_stage_stencil<cdouble, 2>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_stage_stencil<double, 2>), grid, block, 0, s, a);
      break;
    case 3:
      if (c) hipLaunchKernelGGL((k_stage_stencil<cdouble, 3>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_stage_stencil<double, 3>), grid, block, 0, s, a);
      break;
    default:
      return set_error(EXPINT_ENOTSUP, "stencil: d = %d not supported", st.d);
  }
  return check_launch("stage_stencil");
}

int launch_scaled_g(int dtype, long N, const void* U, void* W, double a, int g, double gparam,
                    void* stream) {
  if (N <= 0) return EXPINT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == EXPINT_C128)
    hipLaunchKernelGGL(k_scaled_g<cdouble>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, W, a, g, gparam);
  else
    hipLaunchKernelGGL(k_scaled_g<double>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, W, a, g, gparam);
  return check_launch("scaled_g");
}

int launch_lawson_stage(int dtype, long N, const void* U, void* Wa, void* Wb, double tau, int g,
                        double gparam, void* stream) {
  if (N <= 0) return EXPINT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == EXPINT_C128)
    hipLaunchKernelGGL(k_lawson_stage<cdouble>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, Wa, Wb,
                       tau, g, gparam);
  else
    hipLaunchKernelGGL(k_lawson_stage<double>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, Wa, Wb,
                       tau, g, gparam);
  return check_launch("lawson_stage");
}

}  // namespace expint
