// Exact-slice mu-mode product on int8 MFMA (gfx950).
//
// The mu-mode product (section 1, eq. forloop) is the GEMM
// C[m, q] = sum_k Aop[m, k] Bop[k, q] of the FP64 kernel; here both operands
// are cut into fixed-point digits so that every digit product is exact.
//
// Digits.  A fibre x[0..n) (the values a row of Aop or a column of Bop meets
// along k) gets one power-of-two exponent E with max |x| < 2^(E-1), so
// x' = x 2^-E lies in (-1/2, 1/2).  Six balanced base-128 digits follow by
// repeated rounding: t = 128 x', a = rint(t), x' = t - a (exact in FP64), so
//     x = 2^E sum_{i<6} a_i 128^-(i+1) + r,   a_i in [-64, 64],
//     |r| <= 2^E 128^-6 / 2.
// Digit products a_i b_j are at most 2^12 in magnitude; a level sum of at
// most six of them over k stays exact in int32 for any K below 2^16.
//
// Product.  sum_k x_k y_k = 2^(Ex+Ey) sum_L 128^-(L+2) acc_L with
// acc_L = sum_{i+j=L} sum_k a_i,k b_j,k.  The 26 digit products with
// i + j <= 6 run on int8 MFMA and accumulate exactly in int32; those with
// i + j >= 7 (weight <= 128^-9 per k) are dropped, and the epilogue combines
// the seven level sums in FP64.  With 2^E <= 4 max|x| the error of one
// contraction is at most
//     2^-41 (max|y| sum_k |x_k| + max|x| sum_k |y_k|) + K 2^-44.6 max|x| max|y|
// (digit truncation, then the dropped products), plus FP64 rounding.
//
// Layout.  Digit d of fibre R lives at dig + d * plane + R * Kpad + k, with k
// contiguous and zero-padded to Kpad (a multiple of 64), so an MFMA operand
// fragment (16 consecutive k of one row) is one 16-byte load.
//   mode 1 (s == 1): Aop rows are the rows of M (digits of M along its
//                    columns), Bop columns are the mode-1 fibres of V;
//   mode >= 2:       Aop rows are the mode-mu fibres of V (row b s + m),
//                    Bop columns are the rows of M.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "internal.h"
#include "tile_common.h"

namespace expint {
namespace {

constexpr int kDigits = kSliceDigits;
constexpr int kLevels = kDigits + 1;  // level sums L = i + j = 0 .. kDigits
constexpr int kNonFinite = 1 << 20;  // exponent marking a fibre with inf or nan

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Exponent E with max < 2^(E-1) and the factor 2^-E; a zero fibre gets E = 0.
__device__ __forceinline__ void fibre_exponent(double mx, int* E, double* scale) {
  if (!(mx <= 1.7976931348623157e308)) {  // inf or nan
    *E = kNonFinite;
    *scale = 0.0;
  } else if (mx == 0.0) {
    *E = 0;
    *scale = 0.0;
  } else {
    *E = ilogb(mx) + 2;
    *scale = ldexp(1.0, -*E);
  }
}

// max(mx, |x|) that lets a nan through (fmax would drop it)
__device__ __forceinline__ double absmax(double mx, double x) {
  const double a = fabs(x);
  return (a > mx || a != a) ? a : mx;
}

// Six digits of x' = x 2^-E, one per byte lane `e` of word w[d].
__device__ __forceinline__ void put_digits(double xs, unsigned (&w)[kDigits], int e) {
#pragma unroll
  for (int d = 0; d < kDigits; ++d) {
    const double t = xs * 128.0;
    const double a = __builtin_rint(t);
    xs = t - a;
    w[d] |= ((unsigned)(int)a & 0xffu) << (8 * e);
  }
}

// Fibres along the middle index of a tensor viewed as (s, n, r) with s >= 1:
// x_k = V[m + s k + s n b] for fibre R = b s + m.  A workgroup of 64 x 16
// threads takes 64 consecutive m of one b (lanes along m: coalesced loads);
// thread phase ph holds k = 64 c + 4 ph + e (e < 4) of every 64-wide chunk c
// in registers, so the tensor is read once.  Digits go through an LDS tile
// per chunk and leave as 16-byte pieces: four threads write each 64-byte row
// segment.  Fibres longer than 64 MAXC take k_slice_strided_long.
template <int MAXC>
__global__ __launch_bounds__(1024) void k_slice_strided(const double* __restrict__ V, long s, int n, long r,
                                                        int8_t* __restrict__ dig, long plane,
                                                        int* __restrict__ expo, int Kpad) {
  constexpr int TRS = 68;  // LDS row stride of the digit tile (bytes)
  __shared__ double red[16][64];
  __shared__ __attribute__((aligned(16))) int8_t tile[kDigits][64 * TRS];
  const int lm = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const long mblocks = (s + 63) / 64;
  const long b = blockIdx.x / mblocks;
  const long mbase = (blockIdx.x % mblocks) * 64;
  const long m = mbase + lm;
  const bool valid = m < s;
  const double* f = V + b * s * n + m;
  const int nc = Kpad / 64;
  double x[MAXC][4];
  double mx = 0.0;
#pragma unroll
  for (int c = 0; c < MAXC; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 64 * c + 4 * ph + e;
      x[c][e] = (c < nc && valid && k < n) ? f[(long)k * s] : 0.0;
      mx = absmax(mx, x[c][e]);
    }
  red[ph][lm] = mx;
  __syncthreads();
  mx = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) mx = absmax(mx, red[q][lm]);
  int E;
  double scale;
  fibre_exponent(mx, &E, &scale);
  if (valid && ph == 0) expo[b * s + m] = E;
  const bool finite = E != kNonFinite;
  // rows of this block that exist, and the first row
  const int rows = (int)(s - mbase < 64 ? s - mbase : 64);
  int8_t* out = dig + (b * s + mbase) * Kpad;
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    if (c >= nc) break;
    unsigned w[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; ++d) w[d] = 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) put_digits(finite ? x[c][e] * scale : 0.0, w, e);
    if (c > 0) __syncthreads();  // the previous chunk's tile has been stored
#pragma unroll
    for (int d = 0; d < kDigits; ++d) *reinterpret_cast<unsigned*>(&tile[d][lm * TRS + 4 * ph]) = w[d];
    __syncthreads();
    // 6 digits x 64 rows x 4 pieces of 16 bytes
    for (int t = threadIdx.x; t < kDigits * 256; t += 1024) {
      const int d = t >> 8, row = (t >> 2) & 63, pc = t & 3;
      if (row < rows) {
        const unsigned* src = reinterpret_cast<const unsigned*>(&tile[d][row * TRS + 16 * pc]);
        *reinterpret_cast<uint4*>(out + d * plane + (long)row * Kpad + 64 * c + 16 * pc) =
            make_uint4(src[0], src[1], src[2], src[3]);
      }
    }
  }
}

// Strided fibres of any length: the same mapping, reading the tensor twice
// (once for the exponent, once for the digits).
__global__ __launch_bounds__(256) void k_slice_strided_long(const double* __restrict__ V, long s, int n, long r,
                                                            int8_t* __restrict__ dig, long plane,
                                                            int* __restrict__ expo, int Kpad) {
  const int lm = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const long mblocks = (s + 63) / 64;
  const long b = blockIdx.x / mblocks;
  const long m = (blockIdx.x % mblocks) * 64 + lm;
  const bool valid = m < s;
  const double* f = V + b * s * n + m;
  double mx = 0.0;
  if (valid)
    for (int k = ph; k < n; k += 4) mx = absmax(mx, f[(long)k * s]);
  __shared__ double red[4][64];
  red[ph][lm] = mx;
  __syncthreads();
  mx = absmax(absmax(red[0][lm], red[1][lm]), absmax(red[2][lm], red[3][lm]));
  int E;
  double scale;
  fibre_exponent(mx, &E, &scale);
  if (!valid) return;
  const long R = b * s + m;
  if (ph == 0) expo[R] = E;
  int8_t* row = dig + R * Kpad;
  for (int k0 = 16 * ph; k0 < Kpad; k0 += 64) {
    unsigned w[4][kDigits];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int d = 0; d < kDigits; ++d) w[q][d] = 0u;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int k = k0 + e;
      const double x = (k < n && E != kNonFinite) ? f[(long)k * s] * scale : 0.0;
      put_digits(x, w[e >> 2], e & 3);
    }
#pragma unroll
    for (int d = 0; d < kDigits; ++d)
      *reinterpret_cast<uint4*>(row + d * plane + k0) = make_uint4(w[0][d], w[1][d], w[2][d], w[3][d]);
  }
}

// Contiguous fibres (mode 1): x_k = V[k + n b].  One wave per fibre; lane l
// holds k = 256 c + 4 l + e (e < 4) for the MAXC passes c in registers and
// writes four digits per pass and plane (256 contiguous bytes per wave).
template <int MAXC>
__global__ __launch_bounds__(256) void k_slice_contig(const double* __restrict__ V, int n, long r,
                                                      int8_t* __restrict__ dig, long plane, int* __restrict__ expo,
                                                      int Kpad) {
  const int lane = threadIdx.x & 63;
  const long b = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= r) return;
  const double* f = V + b * n;
  double x[MAXC][4];
  double mx = 0.0;
#pragma unroll
  for (int c = 0; c < MAXC; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = 256 * c + 4 * lane + e;
      x[c][e] = k < n ? f[k] : 0.0;
      mx = absmax(mx, x[c][e]);
    }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = absmax(mx, __shfl_xor(mx, off, 64));
  int E;
  double scale;
  fibre_exponent(mx, &E, &scale);
  if (lane == 0) expo[b] = E;
  const bool finite = E != kNonFinite;
  int8_t* row = dig + b * Kpad;
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    const int k0 = 256 * c + 4 * lane;
    if (k0 >= Kpad) break;
    unsigned w[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; ++d) w[d] = 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) put_digits(finite ? x[c][e] * scale : 0.0, w, e);
#pragma unroll
    for (int d = 0; d < kDigits; ++d) *reinterpret_cast<unsigned*>(row + d * plane + k0) = w[d];
  }
}

// Contiguous fibres of any length (two passes over the fibre).
__global__ __launch_bounds__(256) void k_slice_contig_long(const double* __restrict__ V, int n, long r,
                                                           int8_t* __restrict__ dig, long plane,
                                                           int* __restrict__ expo, int Kpad) {
  const int lane = threadIdx.x & 63;
  const long b = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= r) return;
  const double* f = V + b * n;
  double mx = 0.0;
  for (int k = lane; k < n; k += 64) mx = absmax(mx, f[k]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = absmax(mx, __shfl_xor(mx, off, 64));
  int E;
  double scale;
  fibre_exponent(mx, &E, &scale);
  if (lane == 0) expo[b] = E;
  int8_t* row = dig + b * Kpad;
  for (int k0 = 4 * lane; k0 < Kpad; k0 += 256) {
    unsigned w[kDigits];
#pragma unroll
    for (int d = 0; d < kDigits; ++d) w[d] = 0u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + e;
      put_digits((k < n && E != kNonFinite) ? f[k] * scale : 0.0, w, e);
    }
#pragma unroll
    for (int d = 0; d < kDigits; ++d) *reinterpret_cast<unsigned*>(row + d * plane + k0) = w[d];
  }
}

struct SliceGemmArgs {
  const int8_t* A;  // Aop digits: row m + b * a_rpb
  const int* ea;
  long a_plane, a_rpb;
  const int8_t* B;  // Bop digits: column q + b * b_rpb
  const int* eb;
  long b_plane, b_rpb;
  int Kpad;
  long M, Q;
  long sC, ldc;  // output element (m, q, b) = b sC + m + ldc q
  long batches, tiles_m, tiles_q;
  int m_fastest;  // tile order (tile_coord): Bop holds more data than all of Aop
  Epilogue epi;
};

// One TM x TQ output tile per workgroup of WGM x WGQ waves, each wave one
// 32 x 32 block on v_mfma_i32_32x32x32_i8.  K runs in chunks of 64 staged
// through LDS with a register prefetch of the next chunk.  LDS rows are the
// 64 bytes of one chunk; 16-byte piece p of row r sits at p ^ ((r / 2) mod 4),
// so the 8 lanes an LDS access serves per cycle hit disjoint banks both when
// a thread stores its piece and when a fragment (8 rows, one piece) is read.
// v_mfma_i32_32x32x32_i8(X, Y) takes X[i][16 (l/32) + e] and Y[j][16 (l/32) + e]
// (e < 16) in lane l and leaves sum_k X[i][k] Y[j][k] in lane j + 32 ((i/4) mod 2),
// register 4 (i/8) + (i mod 4); with X = Bop and Y = Aop, 32 consecutive m
// share 32 lanes.
template <int TM, int TQ, int WGM, int WGQ>
__global__ __launch_bounds__(64 * WGM * WGQ, 2) void k_sliced_gemm(SliceGemmArgs g) {
  constexpr int NT = 64 * WGM * WGQ;
  constexpr int D = kDigits;
  constexpr int NL = kLevels;
  constexpr int RS = 64;
  static_assert(TM == 32 * WGM && TQ == 32 * WGQ, "one 32 x 32 block per wave");
  constexpr int AP = TM * 4 / NT, BP = TQ * 4 / NT;  // 16-byte pieces per thread per digit
  static_assert(AP * NT == TM * 4 && BP * NT == TQ * 4, "tile / thread mismatch");
  __shared__ __attribute__((aligned(16))) int8_t As[D][TM * RS];
  __shared__ __attribute__((aligned(16))) int8_t Bs[D][TQ * RS];

  const long nt = g.tiles_m * g.tiles_q * g.batches;
  const long T_ = xcd_remap((long)blockIdx.x, nt);
  const TileCoord tc = tile_coord(T_, g.tiles_m, g.tiles_q, g.m_fastest);
  const long tm = tc.tm, tq = tc.tq, b = tc.b;
  const long m0 = tm * TM, q0 = tq * TQ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % WGM) * 32, wq0 = (wave / WGM) * 32;

  // global -> register staging: piece p of a tile row covers k0 + 16 (p mod 4)
  const unsigned abytes = (unsigned)g.a_plane, bbytes = (unsigned)g.b_plane;
  unsigned avo[AP], bvo[BP];
#pragma unroll
  for (int p = 0; p < AP; ++p) {
    const int piece = tid + p * NT, row = piece >> 2;
    const long m = m0 + row;
    avo[p] = m < g.M ? (unsigned)((m + b * g.a_rpb) * g.Kpad + 16 * (piece & 3)) : 0x80000000u;
  }
#pragma unroll
  for (int p = 0; p < BP; ++p) {
    const int piece = tid + p * NT, row = piece >> 2;
    const long q = q0 + row;
    bvo[p] = q < g.Q ? (unsigned)((q + b * g.b_rpb) * g.Kpad + 16 * (piece & 3)) : 0x80000000u;
  }
  v4i ra[D][AP], rb[D][BP];
  auto gload = [&](int k0) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const __amdgpu_buffer_rsrc_t rsa = make_rsrc(g.A + d * g.a_plane, abytes);
      const __amdgpu_buffer_rsrc_t rsb = make_rsrc(g.B + d * g.b_plane, bbytes);
#pragma unroll
      for (int p = 0; p < AP; ++p)
        ra[d][p] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rsa, (int)avo[p], k0, 0));
#pragma unroll
      for (int p = 0; p < BP; ++p)
        rb[d][p] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rsb, (int)bvo[p], k0, 0));
    }
  };
  auto swz = [](int row, int pc) { return row * RS + 16 * (pc ^ ((row >> 1) & 3)); };
  auto sstore = [&]() {
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int p = 0; p < AP; ++p) {
        const int piece = tid + p * NT;
        *reinterpret_cast<v4i*>(&As[d][swz(piece >> 2, piece & 3)]) = ra[d][p];
      }
#pragma unroll
      for (int p = 0; p < BP; ++p) {
        const int piece = tid + p * NT;
        *reinterpret_cast<v4i*>(&Bs[d][swz(piece >> 2, piece & 3)]) = rb[d][p];
      }
    }
  };

  v16i acc[NL];
#pragma unroll
  for (int L = 0; L < NL; ++L)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[L][e] = 0;

  const int fr = lane & 31, fh = lane >> 5;
  const int nk = g.Kpad / 64;
  gload(0);
  for (int c = 0; c < nk; ++c) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (c + 1 < nk) gload((c + 1) * 64);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      v4i af[D], bf[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        af[i] = *reinterpret_cast<const v4i*>(&As[i][swz(wm0 + fr, 2 * ks + fh)]);
        bf[i] = *reinterpret_cast<const v4i*>(&Bs[i][swz(wq0 + fr, 2 * ks + fh)]);
      }
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D && i + j < NL; ++j)
          acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[j], af[i], acc[i + j], 0, 0, 0);
    }
  }

  // acc[L][r]: m = wm0 + (lane mod 32), q = wq0 + 8 (r / 4) + 4 (lane / 32) + (r mod 4)
  const long cbase = b * g.sC;
  const long m = m0 + wm0 + fr;
  if (m >= g.M) return;
  const int Ea = g.ea[m + b * g.a_rpb];
  epilogue_tile<double>(g.epi, [&](auto&& f) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long q = q0 + wq0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (q >= g.Q) continue;
      const int Eb = g.eb[q + b * g.b_rpb];
      double y = (double)acc[NL - 1][r];
#pragma unroll
      for (int L = NL - 2; L >= 0; --L) y = fma(y, 0.0078125, (double)acc[L][r]);
      y = ldexp(y, Ea + Eb - 14);
      if (Ea >= kNonFinite || Eb >= kNonFinite) y = __builtin_nan("");
      f(cbase + m + g.ldc * q, y);
    }
  });
}

int launch_gemm(SliceGemmArgs& g, hipStream_t st) {
  constexpr int TM = 64, TQ = 64;  // 2 x 2 waves of 32 x 32
  g.tiles_m = (g.M + TM - 1) / TM;
  g.tiles_q = (g.Q + TQ - 1) / TQ;
  g.m_fastest = g.Q > g.M * (g.a_rpb ? g.batches : 1);
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  if (nt <= 0) return EXPINT_OK;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "sliced product: too many tiles (%ld)", nt);
  hipLaunchKernelGGL((k_sliced_gemm<TM, TQ, 2, 2>), dim3((unsigned)nt), dim3(256), 0, st, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "sliced product launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

}  // namespace

int slice_kpad(int n) { return (n + 63) / 64 * 64; }

size_t slice_digits_bytes(long rows, int n) {
  const size_t plane = (size_t)rows * (size_t)slice_kpad(n);
  return ((size_t)kDigits * plane + 255) / 256 * 256 + ((size_t)rows * sizeof(int) + 255) / 256 * 256;
}

int launch_slice(const double* V, long s, int n, long r, bool contiguous, void* out, void* stream) {
  const int Kpad = slice_kpad(n);
  const long rows = s * r;
  const long plane = rows * (long)Kpad;
  if ((size_t)plane >= (1ull << 31)) return set_error(EXPINT_EINVAL, "sliced product: digit plane too large");
  if (n > 65535) return set_error(EXPINT_EINVAL, "sliced product: n = %d exceeds 65535", n);
  int8_t* dig = static_cast<int8_t*>(out);
  int* expo = reinterpret_cast<int*>(dig + ((size_t)kDigits * plane + 255) / 256 * 256);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (rows <= 0) return EXPINT_OK;
  if (contiguous) {
    const long blocks = (r + 3) / 4;
    if (blocks > 0x7fffffffL) return set_error(EXPINT_EINVAL, "sliced product: too many fibres");
    if (Kpad <= 512)
      hipLaunchKernelGGL(k_slice_contig<2>, dim3((unsigned)blocks), dim3(256), 0, st, V, n, r, dig, plane, expo,
                         Kpad);
    else
      hipLaunchKernelGGL(k_slice_contig_long, dim3((unsigned)blocks), dim3(256), 0, st, V, n, r, dig, plane, expo,
                         Kpad);
  } else {
    const long blocks = (s + 63) / 64 * r;
    if (blocks > 0x7fffffffL) return set_error(EXPINT_EINVAL, "sliced product: too many fibres");
    if (Kpad <= 512)
      hipLaunchKernelGGL(k_slice_strided<8>, dim3((unsigned)blocks), dim3(1024), 0, st, V, s, n, r, dig, plane,
                         expo, Kpad);
    else
      hipLaunchKernelGGL(k_slice_strided_long, dim3((unsigned)blocks), dim3(256), 0, st, V, s, n, r, dig, plane,
                         expo, Kpad);
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "slice launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

int launch_sliced_mode_product(long s, int n, long r, bool mode1, const void* Mdig, const void* Vdig,
                               const Epilogue& epi, void* stream) {
  const int Kpad = slice_kpad(n);
  SliceGemmArgs g{};
  const int8_t* md = static_cast<const int8_t*>(Mdig);
  const int8_t* vd = static_cast<const int8_t*>(Vdig);
  const long mplane = (long)n * Kpad;
  const int* mexp = reinterpret_cast<const int*>(md + ((size_t)kDigits * mplane + 255) / 256 * 256);
  const long vrows = s * r;
  const long vplane = vrows * (long)Kpad;
  const int* vexp = reinterpret_cast<const int*>(vd + ((size_t)kDigits * vplane + 255) / 256 * 256);
  g.Kpad = Kpad;
  g.epi = epi;
  if (mode1) {
    // C[i1, q] = sum_k M[i1, k] V[k, q]
    g.A = md, g.ea = mexp, g.a_plane = mplane, g.a_rpb = 0;
    g.B = vd, g.eb = vexp, g.b_plane = vplane, g.b_rpb = 0;
    g.M = n, g.Q = r, g.batches = 1;
    g.sC = 0, g.ldc = n;
  } else {
    // C[m, i_mu] = sum_k V[m, k] M[i_mu, k] for each outer index b
    g.A = vd, g.ea = vexp, g.a_plane = vplane, g.a_rpb = s;
    g.B = md, g.eb = mexp, g.b_plane = mplane, g.b_rpb = 0;
    g.M = s, g.Q = n, g.batches = r;
    g.sC = s * n, g.ldc = s;
  }
  return launch_gemm(g, static_cast<hipStream_t>(stream));
}

}  // namespace expint
