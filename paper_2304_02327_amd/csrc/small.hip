// Fused time stepping for small two-dimensional problems (n1, n2 <= 64).
//
// The state of such a problem is at most 4096 values (32 KB): a whole run of
// many steps fits in one workgroup, with the state and the stage tensors in
// LDS, so the step costs MFMA time instead of kernel launches.  Per step the
// workgroup forms the stage input, applies the split Tucker operator
//     P = W x_1 M_1 x_2 M_2 = M_1 W M_2^T      (U column-major n1 x n2)
// as two 64 x 64 x 64 FP64 MFMA products (one 16 x 16 block per wave), and
// combines the stages as the schemes of section 3.2 prescribe (eq.
// lawsoneulertensor, lawson2tensor, expEulertensor, ETD2RKtensor with the
// split factor (2!)^{d-1} = 2).  Only autonomous g are supported here.
//
// v_mfma_f64_16x16x4 takes A[i][k] in lane i + 16 k and B[k][j] in lane
// j + 16 k and leaves D[i][j] in lane j + 16 (i mod 4), register i / 4.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace expint {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMaxN = 64;
constexpr int kMaxElems = (kMaxN + 1) * kMaxN;  // LDS tensors use an odd leading dimension
constexpr int kThreads = 512;  // 8 waves: one 16 x 32 output strip each

// LDS tensors hold element (i1, i2) at i1 + ld i2 with ld = n1 rounded up to
// an odd number: a column-stride access by 16 lanes then touches 16 distinct
// banks.
struct Lds {
  double U[kMaxElems], W[kMaxElems], X[kMaxElems], T[kMaxElems];
  double cf[2][3][kMaxN];  // stencil coefficients (sub, diag, super) per direction
};

// C = A B (m x q, contraction length kk <= 64).  Wave w owns the 16 x 32
// strip of rows 16 (w mod 4), columns 32 (w / 4): two 16 x 16 blocks that
// share their A operands and run two independent MFMA chains.  a(i, k) and
// b(k, j) return operands, epi(i, j, y) stores.  Operands are loaded in two
// groups of eight k steps ahead of their MFMAs, so a product waits for two
// memory latencies instead of one per k step.
template <typename FA, typename FB, typename FE>
__device__ __forceinline__ void block_gemm(int m, int q, int kk, FA&& a, FB&& b, FE&& epi) {
  constexpr int KI = kMaxN / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bi = (wave & 3) * 16, bj = (wave >> 2) * 32;
  if (bi >= m || bj >= q) return;
  const int r = lane & 15, kq = lane >> 4;
  const bool rowok = bi + r < m, col0 = bj + r < q, col1 = bj + 16 + r < q;
  constexpr int G = KI / 2;  // k steps per prefetch group
  v4d c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int g0 = 0; g0 < KI; g0 += G) {
    if (4 * g0 >= kk) break;
    double av[G], b0[G], b1[G];
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const int k = 4 * (g0 + t) + kq;
      const bool kok = k < kk;
      av[t] = (rowok && kok) ? a(bi + r, k) : 0.0;
      b0[t] = (col0 && kok) ? b(k, bj + r) : 0.0;
      b1[t] = (col1 && kok) ? b(k, bj + 16 + r) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < G; ++t)
      if (4 * (g0 + t) < kk) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], b0[t], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], b1[t], c1, 0, 0, 0);
      }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = bi + 4 * t + kq;
    if (i >= m) continue;
    if (bj + r < q) epi(i, bj + r, c0[t]);
    if (bj + 16 + r < q) epi(i, bj + 16 + r, c1[t]);
  }
}

template <int SCHEME, bool STENCIL>
__global__ __launch_bounds__(kThreads) void k_small2d(SmallArgs a) {
  __shared__ Lds s;
  const int n1 = a.n1, n2 = a.n2, N = n1 * n2;
  const int ld = n1 | 1;
  const int tid = threadIdx.x;
  // logical element e = i1 + n1 i2 of the global tensor -> LDS index
  auto lx = [&](int e) { return e + (ld - n1) * (e / n1); };
  for (int e = tid; e < N; e += kThreads) s.U[lx(e)] = a.U[e];
  if (STENCIL)
    for (int e = tid; e < 3 * (n1 + n2); e += kThreads) {
      const int mu = e < 3 * n1 ? 0 : 1;
      const int o = mu ? e - 3 * n1 : e;
      const int n = mu ? n2 : n1;
      s.cf[mu][o / n][o % n] = a.stc[mu][o];
    }
  __syncthreads();

  const double tau = a.tau, gp = a.gparam;
  const int g = a.g;
  // K U at LDS index x of element (i1, i2) (stencil) -- dense A uses the GEMM below
  auto stencil_ku = [&](int i1, int i2, int x) {
    double v = s.cf[0][1][i1] * s.U[x] + s.cf[1][1][i2] * s.U[x];
    if (i1 > 0) v += s.cf[0][0][i1] * s.U[x - 1];
    else if (a.periodic[0] && n1 > 1) v += s.cf[0][0][0] * s.U[x + n1 - 1];
    if (i1 < n1 - 1) v += s.cf[0][2][i1] * s.U[x + 1];
    else if (a.periodic[0] && n1 > 1) v += s.cf[0][2][n1 - 1] * s.U[x - (n1 - 1)];
    if (i2 > 0) v += s.cf[1][0][i2] * s.U[x - ld];
    else if (a.periodic[1] && n2 > 1) v += s.cf[1][0][0] * s.U[x + ld * (n2 - 1)];
    if (i2 < n2 - 1) v += s.cf[1][2][i2] * s.U[x + ld];
    else if (a.periodic[1] && n2 > 1) v += s.cf[1][2][n2 - 1] * s.U[x - ld * (n2 - 1)];
    return v;
  };
  // W = tau (K U + g(U)); the dense form first puts A_1 U into T
  // elementwise work in 2-D: thread t keeps i1 = t mod 64 and walks i2
  const int ei1 = tid & (kMaxN - 1), ei2 = tid / kMaxN;
  constexpr int kRows = kThreads / kMaxN;
  auto stage_input = [&]() {
    if constexpr (STENCIL) {
      if (ei1 < n1) {
        // at most kMaxN / kRows rows per thread: unrolled so their LDS reads overlap
        double w[kMaxN / kRows];
#pragma unroll
        for (int it = 0; it < kMaxN / kRows; ++it) {
          const int i2 = ei2 + kRows * it;
          if (i2 < n2) {
            const int x = ei1 + ld * i2;
            w[it] = tau * (stencil_ku(ei1, i2, x) + g_eval(g, s.U[x], gp));
          }
        }
#pragma unroll
        for (int it = 0; it < kMaxN / kRows; ++it) {
          const int i2 = ei2 + kRows * it;
          if (i2 < n2) s.W[ei1 + ld * i2] = w[it];
        }
      }
    } else {
      const double* A1 = a.A[0];
      const double* A2 = a.A[1];
      block_gemm(
          n1, n2, n1, [&](int i, int k) { return A1[i + n1 * k]; }, [&](int k, int j) { return s.U[k + ld * j]; },
          [&](int i, int j, double y) { s.T[i + ld * j] = y; });
      __syncthreads();
      // W = tau (A_1 U + U A_2^T + g(U))
      block_gemm(
          n1, n2, n2, [&](int i, int k) { return s.U[i + ld * k]; }, [&](int k, int j) { return A2[j + n2 * k]; },
          [&](int i, int j, double y) {
            const int x = i + ld * j;
            s.W[x] = tau * (s.T[x] + y + g_eval(g, s.U[x], gp));
          });
    }
  };
  // T = M_1 V, then out(x, (T M_2^T)[i, j]) with x the LDS index of (i, j)
  auto tucker = [&](const double* M1, const double* M2, const double* V, auto&& out) {
    block_gemm(
        n1, n2, n1, [&](int i, int k) { return M1[i + n1 * k]; }, [&](int k, int j) { return V[k + ld * j]; },
        [&](int i, int j, double y) { s.T[i + ld * j] = y; });
    __syncthreads();
    block_gemm(
        n1, n2, n2, [&](int i, int k) { return s.T[i + ld * k]; }, [&](int k, int j) { return M2[j + n2 * k]; },
        [&](int i, int j, double y) { out(i + ld * j, y); });
  };
  // elementwise loop over the LDS indices of all elements
  auto each = [&](auto&& f) {
    if (ei1 < n1) {
#pragma unroll
      for (int it = 0; it < kMaxN / kRows; ++it) {
        const int i2 = ei2 + kRows * it;
        if (i2 < n2) f(ei1 + ld * i2);
      }
    }
  };

  for (int step = 0; step < a.nsteps; ++step) {
    switch (SCHEME) {
      case EXPINT_EXP_EULER:
        // U_{n+1} = U_n + (tau (K U_n + G_n)) x phi_1
        stage_input();
        __syncthreads();
        tucker(a.M[0][1], a.M[1][1], s.W, [&](int x, double y) { s.U[x] += y; });
        break;
      case EXPINT_ETD2RK:
        // U_n2 = U_n + (tau (K U_n + G_n)) x phi_1;  W_2 = tau (G(U_n2) - G_n)
        // U_{n+1} = U_n2 + 2 W_2 x phi_2
        stage_input();
        __syncthreads();
        tucker(a.M[0][1], a.M[1][1], s.W, [&](int x, double y) {
          const double u = s.U[x], u2 = u + y;
          s.X[x] = u2;
          s.W[x] = tau * (g_eval(g, u2, gp) - g_eval(g, u, gp));
        });
        __syncthreads();
        tucker(a.M[0][2], a.M[1][2], s.W, [&](int x, double y) { s.U[x] = s.X[x] + 2.0 * y; });
        break;
      case EXPINT_LAWSON_EULER:
        // U_{n+1} = (U_n + tau G_n) x e^{tau A}
        each([&](int x) { s.W[x] = s.U[x] + tau * g_eval(g, s.U[x], gp); });
        __syncthreads();
        tucker(a.M[0][0], a.M[1][0], s.W, [&](int x, double y) { s.U[x] = y; });
        break;
      case EXPINT_LAWSON2B:
        // U_n2 = (U_n + tau G_n) x e^{tau A};  U_{n+1} = (U_n + tau/2 G_n) x e^{tau A} + tau/2 G(U_n2)
        each([&](int x) {
          const double gu = g_eval(g, s.U[x], gp);
          s.W[x] = s.U[x] + tau * gu;
          s.X[x] = s.U[x] + 0.5 * tau * gu;
        });
        __syncthreads();
        tucker(a.M[0][0], a.M[1][0], s.W, [&](int x, double y) { s.W[x] = y; });
        __syncthreads();
        tucker(a.M[0][0], a.M[1][0], s.X, [&](int x, double y) { s.U[x] = y + 0.5 * tau * g_eval(g, s.W[x], gp); });
        break;
      default:
        break;
    }
    __syncthreads();
  }
  for (int e = tid; e < N; e += kThreads) a.U[e] = s.U[lx(e)];
}

}  // namespace

bool small2d_fits(int d, const int* n) {
  return d == 2 && n[0] >= 1 && n[1] >= 1 && n[0] <= kMaxN && n[1] <= kMaxN;
}

int launch_small2d(const SmallArgs& a, void* stream) {
  const int n[2] = {a.n1, a.n2};
  if (!small2d_fits(2, n))
    return set_error(EXPINT_EINVAL, "fused small path: n1 = %d, n2 = %d exceed %d", a.n1, a.n2, kMaxN);
  if (a.nsteps <= 0) return EXPINT_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool sten = a.stencil != 0;
  switch (a.scheme) {
    case EXPINT_EXP_EULER:
      if (sten)
        hipLaunchKernelGGL((k_small2d<EXPINT_EXP_EULER, true>), dim3(1), dim3(kThreads), 0, st, a);
      else
        hipLaunchKernelGGL((k_small2d<EXPINT_EXP_EULER, false>), dim3(1), dim3(kThreads), 0, st, a);
      break;
    case EXPINT_ETD2RK:
      if (sten)
        hipLaunchKernelGGL((k_small2d<EXPINT_ETD2RK, true>), dim3(1), dim3(kThreads), 0, st, a);
      else
        hipLaunchKernelGGL((k_small2d<EXPINT_ETD2RK, false>), dim3(1), dim3(kThreads), 0, st, a);
      break;
    case EXPINT_LAWSON_EULER:
      hipLaunchKernelGGL((k_small2d<EXPINT_LAWSON_EULER, false>), dim3(1), dim3(kThreads), 0, st, a);
      break;
    case EXPINT_LAWSON2B:
      hipLaunchKernelGGL((k_small2d<EXPINT_LAWSON2B, false>), dim3(1), dim3(kThreads), 0, st, a);
      break;
    default:
      return set_error(EXPINT_EINVAL, "fused small path: unknown scheme %d", a.scheme);
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "fused small-problem launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

}  // namespace expint
