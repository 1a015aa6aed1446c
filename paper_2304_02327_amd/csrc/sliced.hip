// Exact-slice mu-mode product on int8 MFMA (gfx950).
//
// The mu-mode product (section 1, eq. forloop) is the GEMM
// C[m, q] = sum_k Aop[m, k] Bop[k, q] of the FP64 kernel; here both operands
// are cut into fixed-point digits so that every digit product is exact.
//
// Digits.  A fibre x[0..n) (the values a row of Aop or a column of Bop meets
// along k) gets one power-of-two exponent E with max |x| < 2^(E-1), so
// x' = x 2^-E lies in (-1/2, 1/2).  Five balanced base-254 digits follow by
// repeated rounding: t = 254 x', a = rint(t), x' = t - a, so
//     x = 2^E (sum_{i<5} a_i 254^-(i+1) + r),   a_i in [-127, 127],
//     |r| <= 254^-5 / 2 + 2^-46.
// |t| <= 127 because |x'| <= 1/2, and t - rint(t) is exact in FP64; only the
// product 254 x' rounds (2^-53 relative, the 2^-46 term above).  A digit
// product is at most 127^2 < 2^14 in magnitude and a level holds at most five
// of them per k, so a level sum over k stays exact in int32 for K <= 26624.
//
// Product.  sum_k x_k y_k = 2^(Ex+Ey) sum_L 254^-(L+2) acc_L with
// acc_L = sum_{i+j=L} sum_k a_i,k b_j,k.  The 19 digit products with
// i + j <= 5 run on int8 MFMA and accumulate exactly in int32; those with
// i + j >= 6 (weight <= 254^-8 per k) are dropped, and the epilogue combines
// the six level sums in FP64 by Horner's rule in powers of 1/254.  With
// 2^E <= 4 max|x| the error of one contraction is at most
//     2^-38.9 (max|y| sum_k |x_k| + max|x| sum_k |y_k|) + K 2^-44.3 max|x| max|y|
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
#include <cstdlib>
#include <cstring>

#include "device_common.h"
#include "internal.h"
#include "tile_common.h"

namespace expint {
namespace {

constexpr int kDigits = kSliceDigits;
constexpr int kLevels = kDigits + 1;  // level sums L = i + j = 0 .. kDigits
constexpr double kBase = 254.0;
constexpr double kInvBase = 1.0 / 254.0;
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

// The digits of x' = x 2^-E, one per byte lane `e` of word w[d].
__device__ __forceinline__ void put_digits(double xs, unsigned (&w)[kDigits], int e) {
#pragma unroll
  for (int d = 0; d < kDigits; ++d) {
    const double t = xs * kBase;
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
// 32 x 32 block on v_mfma_i32_32x32x32_i8.  K runs in chunks of KC bytes per
// row (32 or 64).  Each chunk travels from global memory straight into LDS
// (buffer_load_dwordx4 ... lds: one instruction moves 1 KB, lane l writing
// bytes 16 l .. 16 l + 15 of it), so no registers stage it, into one of S
// stages: while the waves multiply chunk c, chunks c + 1 .. c + S - 2 are in
// flight, and one barrier per chunk both publishes chunk c and frees the stage
// of chunk c - 1 for chunk c + S - 1.  The loads are issued from inline
// assembly, which has no register result (the data goes to LDS at the address
// in M0), so the compiler neither tracks them nor waits for them: the kernel
// counts them itself (vmcnt, in issue order) before each barrier.  In a stage, digit d holds the TM rows of
// Aop and then the TQ rows of Bop, KC bytes each, in 16-byte pieces; piece p of
// row r sits in slot p ^ swizzle(r) (the loading lane picks its piece
// accordingly) with
//     KC = 64: swizzle(r) = ((r / 2) ^ (r / 8)) mod 4,
//     KC = 32: swizzle(r) = ((r / 4) ^ (r / 8)) mod 2,
// so a fragment read (one piece of 32 consecutive rows) hits disjoint banks
// within every 8 lanes (128 bytes) and within every 16 lanes (256 bytes),
// whichever group the LDS serves per cycle.
// v_mfma_i32_32x32x32_i8(X, Y) takes X[i][16 (l/32) + e] and Y[j][16 (l/32) + e]
// (e < 16) in lane l and leaves sum_k X[i][k] Y[j][k] in lane j + 32 ((i/4) mod 2),
// register 4 (i/8) + (i mod 4); with X = Bop and Y = Aop, 32 consecutive m
// share 32 lanes.
template <int WGM, int WGQ, int KC, int S>
struct SliceTile {
  static constexpr int NW = WGM * WGQ;
  static constexpr int TM = 32 * WGM, TQ = 32 * WGQ;
  static constexpr int PR = KC / 16;             // pieces per row
  static constexpr int RPI = 64 / PR;            // rows per DMA instruction
  static constexpr int ROWS = TM + TQ;           // rows of one digit in one stage
  static constexpr int DBYTES = ROWS * KC;       // one digit of one stage
  static constexpr int BBYTES = kDigits * DBYTES;
  static constexpr int RG = ROWS / RPI;          // row groups per digit
  static constexpr int NI = kDigits * RG;        // DMA instructions per chunk
  static constexpr int NIW = (NI + NW - 1) / NW;  // per wave (the last one guarded)
  static constexpr int NIW_MIN = NI / NW;         // issued by every wave
  static_assert(KC == 32 || KC == 64, "chunk of 32 or 64 bytes");
  static_assert(TM % RPI == 0 && TQ % RPI == 0, "row groups");
  static_assert(S >= 2 && S <= 4, "2 to 4 stages");
  static_assert((S - 2) * NIW_MIN <= 63, "vmcnt range");
  __device__ static int swz(int r) {
    return KC == 64 ? (((r >> 1) ^ (r >> 3)) & 3) : (((r >> 2) ^ (r >> 3)) & 1);
  }
};

template <int BYTES>
struct alignas(1024) StageMem {
  int8_t b[BYTES];
};

// One LDS DMA load: 64 lanes x 16 bytes from the buffer `r` at voff + soff to
// LDS bytes [lds, lds + 1024), lane l's at lds + 16 l.  Out-of-range offsets
// read zeros.
__device__ __forceinline__ void dma_b128(__amdgpu_buffer_rsrc_t r, unsigned lds, unsigned voff, int soff) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
               :
               : "s"(lds), "v"(voff), "s"(r), "s"(soff)
               : "memory");
}

template <typename P>
__device__ __forceinline__ unsigned lds_offset(P* p) {
  return (unsigned)(uintptr_t)(__attribute__((address_space(3))) P*)p;
}

template <int WGM, int WGQ, int KC, int S, int OCC>
__global__ __launch_bounds__(64 * WGM * WGQ, OCC) void k_sliced_gemm(SliceGemmArgs g) {
  using T = SliceTile<WGM, WGQ, KC, S>;
  constexpr int NW = T::NW, TM = T::TM, TQ = T::TQ, NL = kLevels, PR = T::PR;
  // one LDS object per stage, so that the compiler sees that reading one stage
  // does not depend on the loads in flight into the others
  __shared__ StageMem<T::BBYTES> st0;
  __shared__ StageMem<T::BBYTES> st1;
  __shared__ StageMem<S >= 3 ? T::BBYTES : 16> st2;
  __shared__ StageMem<S >= 4 ? T::BBYTES : 16> st3;
  auto stage = [&](int i) -> int8_t* {
    return i == 0 ? st0.b : i == 1 ? st1.b : i == 2 ? st2.b : st3.b;
  };

  const long nt = g.tiles_m * g.tiles_q * g.batches;
  const long T_ = xcd_remap((long)blockIdx.x, nt);
  const TileCoord tc = tile_coord(T_, g.tiles_m, g.tiles_q, g.m_fastest);
  const long tm = tc.tm, tq = tc.tq, b = tc.b;
  const long m0 = tm * TM, q0 = tq * TQ;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave % WGM) * 32, wq0 = (wave / WGM) * 32;

  // DMA instruction u of this wave moves row group t mod RG of digit t / RG
  // (t = wave + NW u); its lane l fills slot l mod PR of row RPI (t mod RG) + l / PR
  const unsigned abytes = (unsigned)g.a_plane, bbytes = (unsigned)g.b_plane;
  unsigned voff[T::NIW];
#pragma unroll
  for (int u = 0; u < T::NIW; ++u) {
    const int t = wave + NW * u;
    const int r = T::RPI * (t % T::RG) + lane / PR;
    const int piece = (lane % PR) ^ T::swz(r);
    unsigned o = 0x80000000u;
    if (r < TM) {
      const long m = m0 + r;
      if (m < g.M) o = (unsigned)((m + b * g.a_rpb) * g.Kpad + 16 * piece);
    } else {
      const long q = q0 + (r - TM);
      if (q < g.Q) o = (unsigned)((q + b * g.b_rpb) * g.Kpad + 16 * piece);
    }
    voff[u] = o;
  }
  // DMA instruction u of chunk k0 into stage dst
  auto issue_one = [&](int8_t* dst, int k0, int u) {
    const int t = wave + NW * u;
    if (u < T::NIW_MIN || t < T::NI) {
      const int d = t / T::RG, rg = t % T::RG;
      const bool isa = T::RPI * rg < TM;
      const __amdgpu_buffer_rsrc_t rs =
          isa ? make_rsrc(g.A + d * g.a_plane, abytes) : make_rsrc(g.B + d * g.b_plane, bbytes);
      dma_b128(rs, lds_offset(dst + d * T::DBYTES + rg * 1024), voff[u], k0);
    }
  };
  auto issue = [&](int8_t* dst, int k0) {
#pragma unroll
    for (int u = 0; u < T::NIW; ++u) issue_one(dst, k0, u);
  };

  v16i acc[NL];
#pragma unroll
  for (int L = 0; L < NL; ++L)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[L][e] = 0;

  // fragment byte offsets (k step ks of a chunk): A row wm0 + (lane mod 32),
  // B row TM + wq0 + (lane mod 32), piece 2 ks + lane / 32
  const int fr = lane & 31, fh = lane >> 5;
  auto frag = [](int row, int pc) { return row * KC + 16 * (pc ^ T::swz(row)); };
  int ao[KC / 32], bo[KC / 32];
#pragma unroll
  for (int ks = 0; ks < KC / 32; ++ks) {
    ao[ks] = frag(wm0 + fr, 2 * ks + fh);
    bo[ks] = frag(TM + wq0 + fr, 2 * ks + fh);
  }
  // Multiply the chunk in stage src; when `next` is set, the DMA instructions
  // of the chunk at k0 into stage `next` are spread evenly between the MFMAs
  // (pinned there by scheduling barriers), so that a burst of them does not
  // hold up the MFMAs behind it while the memory pipeline's queue is full.
  constexpr int NMF = (KC / 32) * kSliceProducts;  // MFMAs per chunk
  constexpr int STEP = NMF / T::NIW > 0 ? NMF / T::NIW : 1;
  auto compute = [&](const int8_t* src, int8_t* next, int k0) {
    int t = 0;
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      v4i af[kDigits], bf[kDigits];
#pragma unroll
      for (int i = 0; i < kDigits; ++i) {
        af[i] = *reinterpret_cast<const v4i*>(src + i * T::DBYTES + ao[ks]);
        bf[i] = *reinterpret_cast<const v4i*>(src + i * T::DBYTES + bo[ks]);
      }
#pragma unroll
      for (int i = 0; i < kDigits; ++i)
#pragma unroll
        for (int j = 0; j < kDigits && i + j < NL; ++j) {
          acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(bf[j], af[i], acc[i + j], 0, 0, 0);
          ++t;
          if (t % STEP == 0 && t / STEP <= T::NIW && next) {
            __builtin_amdgcn_sched_barrier(0);
            issue_one(next, k0, t / STEP - 1);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
    }
#pragma unroll
    for (int u = NMF / STEP; u < T::NIW; ++u)
      if (next) issue_one(next, k0, u);
  };
  // chunk c has landed in this wave once at most the loads of the S - 2 chunks
  // issued after it are outstanding (loads complete in order); the barrier then
  // covers every wave
  auto landed = [&]() {
    constexpr int n = (S - 2) * T::NIW_MIN;
    asm volatile("s_waitcnt vmcnt(%0)" : : "n"(n) : "memory");
    __syncthreads();
  };

  const int nk = g.Kpad / KC;
#pragma unroll
  for (int c = 0; c < S - 1; ++c)
    if (c < nk) issue(stage(c), c * KC);
  for (int c0 = 0; c0 < nk; c0 += S) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int c = c0 + u;
      if (c < nk) {
        if (c + S - 2 >= nk) {
          asm volatile("s_waitcnt vmcnt(0)" : : : "memory");  // the tail: fewer chunks after c
          __syncthreads();
        } else {
          landed();
        }
        compute(stage(u), c + S - 1 < nk ? stage((u + S - 1) % S) : nullptr, (c + S - 1) * KC);
      }
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
      for (int L = NL - 2; L >= 0; --L) y = fma(y, kInvBase, (double)acc[L][r]);
      y = ldexp(y * (kInvBase * kInvBase), Ea + Eb);
      if (Ea >= kNonFinite || Eb >= kNonFinite) y = __builtin_nan("");
      f(cbase + m + g.ldc * q, y);
    }
  });
}

// Tile shapes of the sliced product: TMxTQ outputs, w = waves, k = chunk bytes,
// s = stages, o = workgroups per CU.  EXPINT_SLICE_TILE names one to force it.
// Measured at 384^3 (MI355X): 64x64 on 4 waves, two workgroups per CU, is the
// fastest of these (about 550 us per mode product, 30% of the int8 MFMA peak);
// deeper pipelines (3-4 stages of 32-byte chunks) measured slower, since the
// time goes to the volume the memory pipeline moves rather than to its latency.
const char* const kSliceTileNames[] = {"64x64w4k64s2o2", "128x64w8k64s2o1", "64x128w8k64s2o1",
                                       "64x64w4k32s2o3", "64x64w4k32s4o2",  "128x64w8k32s4o1"};
constexpr int kNumSliceTiles = sizeof(kSliceTileNames) / sizeof(kSliceTileNames[0]);

template <int WGM, int WGQ, int KC, int S, int OCC>
int launch_gemm_tile(SliceGemmArgs& g, hipStream_t st) {
  constexpr int TM = 32 * WGM, TQ = 32 * WGQ;
  g.tiles_m = (g.M + TM - 1) / TM;
  g.tiles_q = (g.Q + TQ - 1) / TQ;
  g.m_fastest = g.Q > g.M * (g.a_rpb ? g.batches : 1);
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  if (nt <= 0) return EXPINT_OK;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "sliced product: too many tiles (%ld)", nt);
  hipLaunchKernelGGL((k_sliced_gemm<WGM, WGQ, KC, S, OCC>), dim3((unsigned)nt), dim3(64 * WGM * WGQ), 0, st, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "sliced product launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

// The autotuner's choice (or EXPINT_SLICE_TILE) comes first.
int launch_gemm(SliceGemmArgs& g, hipStream_t st) {
  int choice = tune_choice(TuneKey{TUNE_SLICED, g.M, g.Q, g.Kpad, g.batches});
  if (choice < 0) choice = 0;
  switch (choice) {
    case 1: return launch_gemm_tile<4, 2, 64, 2, 1>(g, st);
    case 2: return launch_gemm_tile<2, 4, 64, 2, 1>(g, st);
    case 3: return launch_gemm_tile<2, 2, 32, 2, 3>(g, st);
    case 4: return launch_gemm_tile<2, 2, 32, 4, 2>(g, st);
    case 5: return launch_gemm_tile<4, 2, 32, 4, 1>(g, st);
    default: return launch_gemm_tile<2, 2, 64, 2, 2>(g, st);
  }
}

}  // namespace


int sliced_tile_count() { return kNumSliceTiles; }
const char* sliced_tile_name(int i) { return i >= 0 && i < kNumSliceTiles ? kSliceTileNames[i] : "?"; }

// the GEMM launch_sliced_mode_product makes (mode 1 when s == 1)
TuneKey sliced_key(long s, int n, long r) {
  if (s == 1) return TuneKey{TUNE_SLICED, n, r, slice_kpad(n), 1};
  return TuneKey{TUNE_SLICED, s, n, slice_kpad(n), r};
}


int launch_slice(const double* V, long s, int n, long r, bool contiguous, void* out, void* stream) {
  const int Kpad = slice_kpad(n);
  const long rows = s * r;
  const long plane = rows * (long)Kpad;
  if ((size_t)plane >= (1ull << 31)) return set_error(EXPINT_EINVAL, "sliced product: digit plane too large");
  if (n > kSliceMaxK) return set_error(EXPINT_EINVAL, "sliced product: n = %d exceeds %d", n, kSliceMaxK);
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
