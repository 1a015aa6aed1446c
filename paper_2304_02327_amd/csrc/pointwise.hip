// Stage-input kernels: the K u action by a 3-point stencil per direction and
// the pointwise nonlinearity g (paper section 3.2: K u_n is applied in tensor
// form as sum_mu U x_mu A_mu, without assembling K).  These kernels are
// bound by HBM traffic: each reads U once (neighbours come from cache) and
// writes its outputs once.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>

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
  double tc[4][3][2];  // Toeplitz values (lo, di, up) per direction
  const void* U;
  void* W;
  double tau;
  int g;
  double gparam;
  GridTime gt;
};

// Workgroups are dealt round-robin over the 8 XCDs.  Remapping block L so that
// XCD x sweeps the x-th contiguous eighth of the tensor keeps the neighbour
// planes of a block in the L2 of the XCD that reads them (without it every
// XCD fetches the planes above and below its own from memory again).
__device__ __forceinline__ unsigned xcd_block(unsigned L, unsigned nb) {
  const unsigned per = nb / 8u;
  if (L >= per * 8u) return L;
  return (L % 8u) * per + L / 8u;
}

// One thread per element.  N < 2^31, so 32-bit index arithmetic is exact; the
// direction count D is a template parameter so the direction loop unrolls.
template <typename T>
__device__ __forceinline__ T tcoef(const double (&v)[2]);
template <>
__device__ __forceinline__ double tcoef<double>(const double (&v)[2]) { return v[0]; }
template <>
__device__ __forceinline__ cdouble tcoef<cdouble>(const double (&v)[2]) { return cdouble{v[0], v[1]}; }

template <typename T, int D, bool TOEP>
__global__ __launch_bounds__(kThreads) void k_stage_stencil(StencilArgs a) {
  const unsigned e = xcd_block(blockIdx.x, gridDim.x) * (unsigned)kThreads + threadIdx.x;
  if (e >= (unsigned)a.N) return;
  const T* U = static_cast<const T*>(a.U);
  const T u = U[e];
  T acc = zero<T>();
  unsigned rem = e, stride = 1;
  int idx[4] = {0, 0, 0, 0};
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
    idx[mu] = (int)i;
    const T* c = static_cast<const T*>(a.coef[mu]);
    const T clo = TOEP ? tcoef<T>(a.tc[mu][0]) : c[i];
    const T cdi = TOEP ? tcoef<T>(a.tc[mu][1]) : c[nm + i];
    const T cup = TOEP ? tcoef<T>(a.tc[mu][2]) : c[2 * nm + i];
    acc = fma_t(cdi, u, acc);
    if (i > 0)
      acc = fma_t(clo, U[e - stride], acc);
    else if (a.periodic[mu])
      acc = fma_t(clo, U[e + (nm - 1) * stride], acc);
    if (i + 1 < nm)
      acc = fma_t(cup, U[e + stride], acc);
    else if (a.periodic[mu])
      acc = fma_t(cup, U[e - (nm - 1) * stride], acc);
    stride *= nm;
  }
  T gu;
  if constexpr (std::is_same<T, double>::value) {
    if (D == 3 && a.g == EXPINT_G_ADR_PAPER)
      gu = adr_paper_g(a.gt, u, clock_time(a.gt, 0.0), idx[0], idx[1], idx[2]);
    else
      gu = g_eval(a.g, u, a.gparam);
  } else {
    gu = g_eval(a.g, u, a.gparam);
  }
  static_cast<T*>(a.W)[e] = scale(add(acc, gu), a.tau);
}

// Real data with n_1 a multiple of V: a thread takes V consecutive elements of
// one i_1 row.  Its row segment and the neighbouring segments along i_2, i_3,
// ... come in as 16-byte vector loads (the tensors are 16-byte aligned and each
// segment starts at an even element), the two i_1 neighbours outside the
// segment as single loads, and W leaves as vector stores: about 2.5x fewer
// memory instructions than one thread per element.  The terms are summed in
// the same order as in k_stage_stencil.
template <int D, bool TOEP, int V>
__global__ __launch_bounds__(kThreads) void k_stage_stencil_v(StencilArgs a) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  static_assert(V % 2 == 0, "segments are whole 16-byte vectors");
  const unsigned groups = (unsigned)(a.N / V);
  const unsigned gi = xcd_block(blockIdx.x, gridDim.x) * (unsigned)kThreads + threadIdx.x;
  if (gi >= groups) return;
  const unsigned e0 = gi * V;
  const double* U = static_cast<const double*>(a.U);
  auto seg = [&](unsigned at, double (&out)[V]) {
#pragma unroll
    for (int h = 0; h < V / 2; ++h) {
      const v2d t = *reinterpret_cast<const v2d*>(U + at + 2 * h);
      out[2 * h] = t[0];
      out[2 * h + 1] = t[1];
    }
  };
  double u[V], acc[V];
  seg(e0, u);
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = 0.0;
  // direction 1: neighbours inside the segment, plus one on either side
  const unsigned n1 = (unsigned)a.n[0];
  const unsigned i1 = e0 % n1;
  unsigned rem = e0 / n1;
  int idx[4] = {(int)i1, 0, 0, 0};
  {
    const double* c = static_cast<const double*>(a.coef[0]);
    const bool has_lo = i1 > 0 || a.periodic[0], has_up = i1 + V < n1 || a.periodic[0];
    const double left = i1 > 0 ? U[e0 - 1] : (a.periodic[0] ? U[e0 + n1 - 1] : 0.0);
    const double right = i1 + V < n1 ? U[e0 + V] : (a.periodic[0] ? U[e0 + V - n1] : 0.0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double clo = TOEP ? a.tc[0][0][0] : c[i1 + v];
      const double cdi = TOEP ? a.tc[0][1][0] : c[n1 + i1 + v];
      const double cup = TOEP ? a.tc[0][2][0] : c[2 * n1 + i1 + v];
      acc[v] = fma(cdi, u[v], acc[v]);
      if (v > 0) acc[v] = fma(clo, u[v - 1], acc[v]);
      else if (has_lo) acc[v] = fma(clo, left, acc[v]);
      if (v < V - 1) acc[v] = fma(cup, u[v + 1], acc[v]);
      else if (has_up) acc[v] = fma(cup, right, acc[v]);
    }
  }
  unsigned stride = n1;
#pragma unroll
  for (int mu = 1; mu < D; ++mu) {
    const unsigned nm = (unsigned)a.n[mu];
    unsigned i;
    if (mu < D - 1) {
      i = rem % nm;
      rem /= nm;
    } else {
      i = rem;
    }
    idx[mu] = (int)i;
    const double* c = static_cast<const double*>(a.coef[mu]);
    const double clo = TOEP ? a.tc[mu][0][0] : c[i];
    const double cdi = TOEP ? a.tc[mu][1][0] : c[nm + i];
    const double cup = TOEP ? a.tc[mu][2][0] : c[2 * nm + i];
    double lo[V], up[V];
    const bool has_lo = i > 0 || a.periodic[mu], has_up = i + 1 < nm || a.periodic[mu];
    if (has_lo) seg(i > 0 ? e0 - stride : e0 + (nm - 1) * stride, lo);
    if (has_up) seg(i + 1 < nm ? e0 + stride : e0 - (nm - 1) * stride, up);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[v] = fma(cdi, u[v], acc[v]);
      if (has_lo) acc[v] = fma(clo, lo[v], acc[v]);
      if (has_up) acc[v] = fma(cup, up[v], acc[v]);
    }
    stride *= nm;
  }
  double w[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double gu;
    if (D == 3 && a.g == EXPINT_G_ADR_PAPER)
      gu = adr_paper_g(a.gt, u[v], clock_time(a.gt, 0.0), idx[0] + v, idx[1], idx[2]);
    else
      gu = g_eval(a.g, u[v], a.gparam);
    w[v] = (acc[v] + gu) * a.tau;
  }
  double* W = static_cast<double*>(a.W);
#pragma unroll
  for (int h = 0; h < V / 2; ++h) *reinterpret_cast<v2d*>(W + e0 + 2 * h) = v2d{w[2 * h], w[2 * h + 1]};
}

// Three directions, real data, n_1 a multiple of 64 and n_2 of 8: a 2.5-D
// stencil.  A workgroup owns a 64 x 8 tile of (i_1, i_2) and a run of cz planes
// i_3 = k0 .. k1 - 1, and streams along i_3.  A thread holds two consecutive
// i_1 elements of one tile row and keeps their planes k - 1, k and k + 1 in
// registers (the i_3 neighbours); plane k with a one-element halo in i_1 and
// i_2 sits in LDS (the i_1 and i_2 neighbours), two buffers, one barrier per
// plane.  So each element comes from memory once per workgroup (the halo rows
// and columns, which the neighbouring tiles own, come mostly from L2), and
// plane k + 2 is requested while plane k is computed.  Each element's terms are
// summed in the same order as in k_stage_stencil, so the result is the same.
constexpr int kS25X = 64, kS25Y = 8, kS25Z = 32;
template <bool TOEP>
__global__ __launch_bounds__(kThreads) void k_stage_stencil_25d(StencilArgs a, int cz) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  static_assert(kS25X * kS25Y == 2 * kThreads, "two elements per thread");
  constexpr int LX = kS25X + 2, LY = kS25Y + 2;
  constexpr int NH = 2 * kS25X + 2 * kS25Y;  // halo cells of a plane
  __shared__ double buf[2][LY * LX];
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int ntx = n1 / kS25X, nty = n2 / kS25Y;
  const int b = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
  const int x0 = tx * kS25X, y0 = ty * kS25Y;
  const int k0 = tz * cz, k1 = min(n3, k0 + cz);
  const int tid = threadIdx.x, lx = (tid & 31) * 2, ly = tid >> 5;
  const int i1 = x0 + lx, i2 = y0 + ly;
  const long plane = (long)n1 * n2;
  const long orow = (long)i1 + (long)n1 * i2;
  const bool per1 = a.periodic[0], per2 = a.periodic[1], per3 = a.periodic[2];
  const double* U = static_cast<const double*>(a.U);
  // plane k with the periodic wrap, or -1 past either end
  auto pk = [&](int k) { return k < 0 ? (per3 ? k + n3 : -1) : (k >= n3 ? (per3 ? k - n3 : -1) : k); };
  auto load_own = [&](int k, double (&v)[2]) {
    const int kk = pk(k);
    if (kk >= 0) {
      const v2d t = *reinterpret_cast<const v2d*>(U + orow + plane * kk);
      v[0] = t[0];
      v[1] = t[1];
    } else {
      v[0] = 0.0;
      v[1] = 0.0;
    }
  };
  // halo cell of this thread: the rows above and below the tile, the columns
  // left and right of it (none, or the periodic image, past the domain)
  int hpos = -1;
  long hoff = -1;
  if (tid < NH) {
    int yy, xx;
    if (tid < kS25X) {
      yy = 0;
      xx = tid + 1;
    } else if (tid < 2 * kS25X) {
      yy = LY - 1;
      xx = tid - kS25X + 1;
    } else {
      const int c = tid - 2 * kS25X;
      yy = c % kS25Y + 1;
      xx = c < kS25Y ? 0 : LX - 1;
    }
    int g1 = x0 + xx - 1, g2 = y0 + yy - 1;
    bool ok = true;
    if (g1 < 0 || g1 >= n1) {
      ok = per1;
      g1 = g1 < 0 ? g1 + n1 : g1 - n1;
    }
    if (g2 < 0 || g2 >= n2) {
      ok = ok && per2;
      g2 = g2 < 0 ? g2 + n2 : g2 - n2;
    }
    hpos = yy * LX + xx;
    if (ok) hoff = (long)g1 + (long)n1 * g2;
  }
  auto load_halo = [&](int k) -> double {
    const int kk = pk(k);
    return (hoff >= 0 && kk >= 0) ? U[hoff + plane * kk] : 0.0;
  };
  const int me = (ly + 1) * LX + lx + 1;  // LDS position of the first own element
  double p0[2], p1[2], p2[2], q[2];
  load_own(k0 - 1, p0);
  load_own(k0, p1);
  load_own(k0 + 1, p2);
  const double h0 = load_halo(k0);
  double h1 = load_halo(k0 + 1);
  buf[0][me] = p1[0];
  buf[0][me + 1] = p1[1];
  if (hpos >= 0) buf[0][hpos] = h0;
  __syncthreads();
  const double* c1 = static_cast<const double*>(a.coef[0]);
  const double* c2 = static_cast<const double*>(a.coef[1]);
  const double* c3 = static_cast<const double*>(a.coef[2]);
  const bool lo2 = i2 > 0 || per2, up2 = i2 + 1 < n2 || per2;
  const double clo2 = TOEP ? a.tc[1][0][0] : c2[i2];
  const double cdi2 = TOEP ? a.tc[1][1][0] : c2[n2 + i2];
  const double cup2 = TOEP ? a.tc[1][2][0] : c2[2 * n2 + i2];
  const bool adr = a.g == EXPINT_G_ADR_PAPER;  // the only g that reads the device clock
  const double now = adr ? clock_time(a.gt, 0.0) : 0.0;
  double* W = static_cast<double*>(a.W);
  for (int k = k0; k < k1; ++k) {
    const int cb = (k - k0) & 1;
    load_own(k + 2, q);
    const double hq = load_halo(k + 2);
    const double* L = buf[cb];
    const bool lo3 = k > 0 || per3, up3 = k + 1 < n3 || per3;
    const double clo3 = TOEP ? a.tc[2][0][0] : c3[k];
    const double cdi3 = TOEP ? a.tc[2][1][0] : c3[n3 + k];
    const double cup3 = TOEP ? a.tc[2][2][0] : c3[2 * n3 + k];
    double w[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int j1 = i1 + v;
      const double clo = TOEP ? a.tc[0][0][0] : c1[j1];
      const double cdi = TOEP ? a.tc[0][1][0] : c1[n1 + j1];
      const double cup = TOEP ? a.tc[0][2][0] : c1[2 * n1 + j1];
      const double u = p1[v];
      double acc = fma(cdi, u, 0.0);
      if (j1 > 0 || per1) acc = fma(clo, L[me + v - 1], acc);
      if (j1 + 1 < n1 || per1) acc = fma(cup, L[me + v + 1], acc);
      acc = fma(cdi2, u, acc);
      if (lo2) acc = fma(clo2, L[me + v - LX], acc);
      if (up2) acc = fma(cup2, L[me + v + LX], acc);
      acc = fma(cdi3, u, acc);
      if (lo3) acc = fma(clo3, p0[v], acc);
      if (up3) acc = fma(cup3, p2[v], acc);
      const double gu = adr ? adr_paper_g(a.gt, u, now, j1, i2, k) : g_eval(a.g, u, a.gparam);
      w[v] = (acc + gu) * a.tau;
    }
    *reinterpret_cast<v2d*>(W + orow + plane * k) = v2d{w[0], w[1]};
    if (k + 1 < k1) {
      double* N = buf[cb ^ 1];
      N[me] = p2[0];
      N[me + 1] = p2[1];
      if (hpos >= 0) N[hpos] = h1;
      __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      p0[v] = p1[v];
      p1[v] = p2[v];
      p2[v] = q[v];
    }
    h1 = hq;
  }
}

// The 2.5-D stencil's run of planes per workgroup, or 0 where it does not apply
// (it needs enough workgroups to fill the chip: at least four per CU).
int stencil_25d_planes(const Stencil& st, int dtype) {
  if (const char* e = std::getenv("EXPINT_STENCIL25"); e && std::strcmp(e, "0") == 0) return 0;
  if (dtype != EXPINT_F64 || st.d != 3 || st.n[0] % kS25X != 0 || st.n[1] % kS25Y != 0) return 0;
  const long tiles = (long)(st.n[0] / kS25X) * (st.n[1] / kS25Y);
  const int cz = kS25Z;
  const long wgs = tiles * ((st.n[2] + cz - 1) / cz);
  if (const char* e = std::getenv("EXPINT_STENCIL25"); e && std::strcmp(e, "1") == 0) return cz;  // forced
  return wgs >= 1024 ? cz : 0;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scaled_g(long N, const void* Uv, void* Wv, double s,
                                                       int g, double gp, GridTime gt) {
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  if (e >= N) return;
  static_cast<T*>(Wv)[e] = scale(g_at(g, static_cast<const T*>(Uv)[e], gp, gt, e, 0.0), s);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_lawson_stage(long N, const void* Uv, void* Wa, void* Wb,
                                                           double tau, int g, double gp, GridTime gt) {
  const long e = (long)blockIdx.x * kThreads + threadIdx.x;
  if (e >= N) return;
  const T u = static_cast<const T*>(Uv)[e];
  const T gu = g_at(g, u, gp, gt, e, 0.0);
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
                         int g, double gparam, const GridTime& gt, void* stream) {
  if (N <= 0) return EXPINT_OK;
  StencilArgs a;
  a.N = N;
  a.d = st.d;
  for (int mu = 0; mu < 4; ++mu) {
    a.n[mu] = st.n[mu];
    a.periodic[mu] = st.periodic[mu];
    a.coef[mu] = st.coef[mu];
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 2; ++c) a.tc[mu][k][c] = st.tc[mu][k][c];
  }
  a.U = U;
  a.W = W;
  a.tau = tau;
  a.g = g;
  a.gparam = gparam;
  a.gt = gt;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(blocks_for(N)), block(kThreads);
  const bool c = dtype == EXPINT_C128;
#define EXPINT_STENCIL_LAUNCH(D)                                                                     \
  if (st.toeplitz) {                                                                                 \
    if (c) hipLaunchKernelGGL((k_stage_stencil<cdouble, D, true>), grid, block, 0, s, a);           \
    else hipLaunchKernelGGL((k_stage_stencil<double, D, true>), grid, block, 0, s, a);              \
  } else {                                                                                           \
    if (c) hipLaunchKernelGGL((k_stage_stencil<cdouble, D, false>), grid, block, 0, s, a);          \
    else hipLaunchKernelGGL((k_stage_stencil<double, D, false>), grid, block, 0, s, a);             \
  }
  // three directions, n_1 a multiple of 64, n_2 of 8, large enough: the 2.5-D kernel
  if (const int cz = stencil_25d_planes(st, dtype); cz > 0) {
    const long tiles = (long)(st.n[0] / kS25X) * (st.n[1] / kS25Y) * ((st.n[2] + cz - 1) / cz);
    if (st.toeplitz)
      hipLaunchKernelGGL((k_stage_stencil_25d<true>), dim3((unsigned)tiles), block, 0, s, a, cz);
    else
      hipLaunchKernelGGL((k_stage_stencil_25d<false>), dim3((unsigned)tiles), block, 0, s, a, cz);
    return check_launch("stage_stencil_25d");
  }
  // real data with n_1 a multiple of 4 (or 2): the vectorised kernel
  const int V = c ? 1 : (st.n[0] % 4 == 0 ? 4 : (st.n[0] % 2 == 0 ? 2 : 1));
  if (V > 1) {
    const dim3 vgrid(blocks_for(N / V));
#define EXPINT_STENCIL_V(D)                                                                        \
  if (st.toeplitz) {                                                                                \
    if (V == 4) hipLaunchKernelGGL((k_stage_stencil_v<D, true, 4>), vgrid, block, 0, s, a);        \
    else hipLaunchKernelGGL((k_stage_stencil_v<D, true, 2>), vgrid, block, 0, s, a);               \
  } else {                                                                                          \
    if (V == 4) hipLaunchKernelGGL((k_stage_stencil_v<D, false, 4>), vgrid, block, 0, s, a);       \
    else hipLaunchKernelGGL((k_stage_stencil_v<D, false, 2>), vgrid, block, 0, s, a);              \
  }
    switch (st.d) {
      case 1:
        EXPINT_STENCIL_V(1);
        break;
      case 2:
        EXPINT_STENCIL_V(2);
        break;
      case 3:
        EXPINT_STENCIL_V(3);
        break;
      case 4:
        EXPINT_STENCIL_V(4);
        break;
      default:
        return set_error(EXPINT_ENOTSUP, "stencil: d = %d not supported", st.d);
    }
#undef EXPINT_STENCIL_V
    return check_launch("stage_stencil_v");
  }
  switch (st.d) {
    case 1:
      EXPINT_STENCIL_LAUNCH(1);
      break;
    case 2:
      EXPINT_STENCIL_LAUNCH(2);
      break;
    case 3:
      EXPINT_STENCIL_LAUNCH(3);
      break;
    case 4:
      EXPINT_STENCIL_LAUNCH(4);
      break;
    default:
      return set_error(EXPINT_ENOTSUP, "stencil: d = %d not supported", st.d);
  }
#undef EXPINT_STENCIL_LAUNCH
  return check_launch("stage_stencil");
}

int launch_scaled_g(int dtype, long N, const void* U, void* W, double a, int g, double gparam,
                    const GridTime& gt, void* stream) {
  if (N <= 0) return EXPINT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == EXPINT_C128)
    hipLaunchKernelGGL(k_scaled_g<cdouble>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, W, a, g, gparam, gt);
  else
    hipLaunchKernelGGL(k_scaled_g<double>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, W, a, g, gparam, gt);
  return check_launch("scaled_g");
}

int launch_lawson_stage(int dtype, long N, const void* U, void* Wa, void* Wb, double tau, int g,
                        double gparam, const GridTime& gt, void* stream) {
  if (N <= 0) return EXPINT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == EXPINT_C128)
    hipLaunchKernelGGL(k_lawson_stage<cdouble>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, Wa, Wb,
                       tau, g, gparam, gt);
  else
    hipLaunchKernelGGL(k_lawson_stage<double>, dim3(blocks_for(N)), dim3(kThreads), 0, s, N, U, Wa, Wb,
                       tau, g, gparam, gt);
  return check_launch("lawson_stage");
}

namespace {
__global__ void k_clock_set(double* clock, double t0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clock[0] = t0;
    clock[1] = 0.0;
  }
}
__global__ void k_clock_tick(double* clock) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clock[1] += 1.0;
}
}  // namespace

int launch_clock_set(double* clock, double t0, void* stream) {
  hipLaunchKernelGGL(k_clock_set, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), clock, t0);
  return check_launch("clock_set");
}

int launch_clock_tick(double* clock, void* stream) {
  hipLaunchKernelGGL(k_clock_tick, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream), clock);
  return check_launch("clock_tick");
}

// Non-finite check: sets flag[0] |= 1 if any of the `count` doubles is inf or
// nan.  A wave that sees one issues a single atomic; no other write happens,
// so the flag keeps what earlier checks left until the host clears it.
namespace {
__global__ __launch_bounds__(256) void k_finite_check(const double* __restrict__ x, long count, int* flag) {
  bool bad = false;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double v = x[i];
    bad |= !(fabs(v) <= 1.7976931348623157e308);
  }
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
}  // namespace

int launch_finite_check(const double* x, long count, int* flag, void* stream) {
  if (count <= 0) return EXPINT_OK;
  long blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_finite_check, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), x,
                     count, flag);
  return check_launch("finite_check");
}

}  // namespace expint
