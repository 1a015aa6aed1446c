// Device helpers shared by the GEMM-shaped kernels: the XCD-aware tile
// order, buffer resources and the fused epilogue of a mu-mode product.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace expint {

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tile indices so that tiles that share an Aop block
// (consecutive q-tiles) share that XCD's L2.
__device__ __forceinline__ long xcd_remap(long L, long nt) {
  constexpr long X = 8;
  const long per = nt / X;
  if (L >= per * X) return L;
  return (L % X) * per + L / X;
}

// Coordinates (M tile, Q tile, batch) of tile t.  Neighbouring indices, which
// xcd_remap keeps on one XCD and dispatches together, share a panel of the
// larger operand, so its second reader finds it in that XCD's L2: with
// m_fastest (Bop larger than all of Aop, as the tensor in a mode-1 product)
// the M tile runs fastest and neighbours share a Bop panel; otherwise the Q
// tile runs fastest and they share an Aop panel.
struct TileCoord {
  long tm, tq, b;
};
__device__ __forceinline__ TileCoord tile_coord(long t, long tiles_m, long tiles_q, int m_fastest) {
  const long mq = tiles_m * tiles_q;
  const long r = t % mq;
  if (m_fastest) return {r % tiles_m, r / tiles_m, t / mq};
  return {r / tiles_q, r % tiles_q, t / mq};
}

template <typename T>
__device__ __forceinline__ T ld(const void* p, long i) { return static_cast<const T*>(p)[i]; }

// Non-temporal store of a plain product (alpha Y, the intermediate tensors of
// a Tucker chain and tucker_apply's output).  Measured on MI355X at 128^3: a
// plain launch takes 15.6 instead of 16.7 us and an ETD2RK step 121 instead of
// 125 us; the same stores on the stage outputs (U, U_n2, W_2), which the next
// stage reads back at once, made the step slower (128 us), so those stay
// ordinary stores.
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(cdouble* p, cdouble v) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2d{v.re, v.im}, reinterpret_cast<v2d*>(p));
}

// Applies the epilogue to the outputs a thread owns: visit(f) calls f(e, y)
// for each of them.  The op and the nonlinearity are uniform per launch, so
// they are dispatched once, outside the element loop: every path is a short
// loop of its own and the code a launch runs stays compact.
template <typename T, typename Visit>
__device__ __forceinline__ void epilogue_tile(const Epilogue& ep, Visit&& visit) {
  T* out0 = static_cast<T*>(ep.out0);
  switch (ep.op) {
    case EPI_AXPBY:
      if (ep.beta != 0.0)
        visit([&](long e, T y) { out0[e] = add(scale(y, ep.alpha), scale(out0[e], ep.beta)); });
      else
        visit([&](long e, T y) { st_stream(&out0[e], scale(y, ep.alpha)); });
      break;
    case EPI_EXP_EULER:
      visit([&](long e, T y) { out0[e] = add(ld<T>(ep.in1, e), y); });
      break;
    case EPI_ETD2RK_1:
      // U_n2 = U_n + Y and W_2 = tau (g(t_{n+1}, U_n2) - g(t_n, U_n))
      dispatch_g(ep, T{}, [&](const auto& G) {
        const auto g1 = G.at(ep.tau);
        const auto g0 = G.at(0.0);
        T* out1 = static_cast<T*>(ep.out1);
        visit([&](long e, T y) {
          const T u = ld<T>(ep.in1, e);
          const T u2 = add(u, y);
          out0[e] = u2;
          out1[e] = scale(sub(g1(u2, e), g0(u, e)), ep.tau);
        });
      });
      break;
    case EPI_ETD2RK_2:
      visit([&](long e, T y) { out0[e] = add(ld<T>(ep.in1, e), scale(y, ep.c)); });
      break;
    case EPI_LAWSON2B_2:  // U_{n+1} = Y + tau/2 g(t_{n+1}, U_n2)
      dispatch_g(ep, T{}, [&](const auto& G) {
        const auto g1 = G.at(2.0 * ep.c);
        visit([&](long e, T y) { out0[e] = add(y, scale(g1(ld<T>(ep.in1, e), e), ep.c)); });
      });
      break;
    case EPI_DIAG: {
      // square matrix outputs of at most 4096^2 elements: 32-bit index arithmetic
      const unsigned ld = (unsigned)ep.ldiag;
      visit([&](long e, T y) {
        T v = scale(y, ep.alpha);
        if ((unsigned)e % ld == 0u) v = add(v, real_value<T>(ep.c));
        out0[e] = v;
      });
      break;
    }
    case EPI_LINEAR:
      visit([&](long e, T y) {
        T v = scale(y, ep.alpha);
        if (ep.in1) v = add(v, scale(ld<T>(ep.in1, e), ep.beta));
        if (ep.in2) v = add(v, scale(ld<T>(ep.in2, e), ep.c));
        out0[e] = v;
      });
      break;
    default:
      break;
  }
}

// A buffer resource over [p, p + bytes): loads outside the range return zero
// without touching memory.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const T* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)bytes, 0x00020000);
}

}  // namespace expint
