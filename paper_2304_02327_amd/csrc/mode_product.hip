// mu-mode product on FP64 MFMA (gfx950).
//
// The mu-mode product (section 1, eq. forloop):
//     (V x_mu M)[i_1..i_mu..i_d] = sum_j M[i_mu, j] V[i_1..j..i_d].
// With the tensor viewed as (s, n, r) -- s = n_1..n_{mu-1} (stride 1),
// n = n_mu, r = n_{mu+1}..n_d -- it is a GEMM C[m, q] = sum_k Aop[m, k] Bop[k, q]:
//   mode 1 (s == 1): m = i_1, q = the other indices;  Aop = M, Bop = V (k fastest)
//   mode >= 2:       m = the s-index, q = i_mu, one GEMM per outer index;
//                    Aop = V slab (m fastest), Bop = M^T (q fastest).
// Either way Aop and the output have m as the stride-1 index, so loads and
// stores run along contiguous memory (the non-contiguous mode is the K loop).
//
// Tiling: a workgroup of WGM x WGQ wave64s (4 or 8) owns a TM x TQ output
// tile and walks K in chunks of KC, double-buffered in LDS with register
// prefetch of the next chunks.  Each wave owns a (TM/WGM) x (TQ/WGQ) sub-tile
// made of 16x16 MFMA blocks.  v_mfma_f64_16x16x4 leaves D[i][j] in lane j + 16 (i mod 4),
// register i / 4; the B-chunk fragment is passed as the instruction's first
// operand so that 16 consecutive output rows m land in 16 consecutive lanes
// (128-byte store segments).  The last mode's epilogue fuses the stage
// combination and the next stage's g.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "internal.h"
#include "tile_common.h"

namespace expint {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

struct GemmArgs {
  const void* A;  // Aop[m, k] = A[m + lda k] (+ batch * sA)
  long lda;
  const void* B;  // Bop[k, q] = B[k bk + q bq]
  long bk, bq;
  long M, Q, K;
  long sA, sC;  // batch strides of A and of the output tensors
  long ldc;     // output element (m, q, batch) = batch * sC + m + ldc q
  long batches, tiles_m, tiles_q;
  Epilogue epi;
  const int* gate = nullptr;  // grouped launches: tiles run only while *gate > gate_level
  int gate_level = 0;
  int m_fastest = 0;  // tile order, set with the tile counts (tile_coord)
  int cls = 0;        // grouped launches: tile class (0 small, 1 large) and its tile shape
  int tile_m = 64, tile_q = 64;
};

// Bop is shared by all batches, Aop only when sA == 0: the M tile runs fastest
// when Bop holds more data than all of Aop.
static void set_tile_counts(GemmArgs& g, long TM, long TQ) {
  g.tiles_m = (g.M + TM - 1) / TM;
  g.tiles_q = (g.Q + TQ - 1) / TQ;
  g.m_fastest = g.Q > g.M * (g.sA ? g.batches : 1);
}

// Buffer loads: a resource covers exactly one operand (matrix, slab or whole
// tensor), so a read past its end returns zero in hardware.  A K index past
// the end always lands past the end of the operand's range (the operands are
// K-major beyond their last K row), and rows or columns past M or Q are sent
// there explicitly through an out-of-range offset computed once per thread.
// The per-chunk advance along K is a scalar offset.
template <typename T>
__device__ __forceinline__ T buffer_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double buffer_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ cdouble buffer_ld<cdouble>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cdouble, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}

// LDS of one tile: two buffers of the A chunk (KC x TM) and of the B chunk
// (KC x TQ, padded by one column when stored transposed), per real plane.
template <typename T, bool BK, int TM, int TQ, int KC>
constexpr int tile_lds_doubles() {
  return 2 * (std::is_same<T, cdouble>::value ? 2 : 1) * KC * (TM + (BK ? TQ + 1 : TQ));
}

// The LDS of a kernel's tiles: every tile function of one kernel that names the
// same size shares one allocation (tile classes of the grouped launch).
template <int N>
__shared__ double lds_pool[N];

// One TM x TQ output tile (tile index T_ in [0, tiles_m tiles_q batches)) of the
// GEMM described by g, computed by the whole workgroup in lds_pool<LDSN>
// (at least tile_lds_doubles entries).  Used by the single launch below and by
// the grouped launch, whose tile classes share one LDS allocation.
// IL: in the steady-state loop each chunk's MFMAs are interleaved with its LDS
// reads, LDS writes and global loads (scheduling groups) instead of the
// compiler's own order.
template <typename T, bool BK, int TM, int TQ, int KC, int WGM, int WGQ, int PF = 2,
          int LDSN = tile_lds_doubles<T, BK, TM, TQ, KC>(), bool IL = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, long T_) {
  constexpr bool CPLX = std::is_same<T, cdouble>::value;
  constexpr int NP = CPLX ? 2 : 1;                  // real planes per element
  constexpr int NT = 64 * WGM * WGQ;                // threads
  constexpr unsigned SZ = sizeof(T);
  constexpr int LDA_S = TM;                         // LDS row stride of the A chunk
  constexpr int LDB_S = BK ? TQ + 1 : TQ;           // padded when stored transposed
  constexpr int WM = TM / WGM, WQ = TQ / WGQ;
  constexpr int FM = WM / 16, FQ = WQ / 16;
  constexpr int AL = TM * KC / NT, BL = TQ * KC / NT;
  static_assert(AL * NT == TM * KC && BL * NT == TQ * KC, "tile / thread mismatch");
  static_assert(FM >= 1 && FQ >= 1 && WM % 16 == 0 && WQ % 16 == 0 && KC % 4 == 0, "bad tile");

  static_assert(LDSN >= tile_lds_doubles<T, BK, TM, TQ, KC>(), "LDS pool too small");
  // A chunk buffer b, plane p at lds_pool[(b NP + p) KC LDA_S], the B chunks after all of them
  auto As = [](int b, int p, int i) -> double& { return lds_pool<LDSN>[(b * NP + p) * (KC * LDA_S) + i]; };
  auto Bs = [](int b, int p, int i) -> double& {
    return lds_pool<LDSN>[2 * NP * KC * LDA_S + (b * NP + p) * (KC * LDB_S) + i];
  };

  const TileCoord tc = tile_coord(T_, g.tiles_m, g.tiles_q, g.m_fastest);
  const long tm = tc.tm, tq = tc.tq, b = tc.b;
  const int m0 = (int)(tm * TM), q0 = (int)(tq * TQ);
  const int Mi = (int)g.M, Qi = (int)g.Q, Ki = (int)g.K;
  const unsigned lda = (unsigned)g.lda, bk = (unsigned)g.bk, bq = (unsigned)g.bq;

  // operand ranges: Aop = one slab (or M), Bop = M (or the whole tensor)
  const T* A = static_cast<const T*>(g.A) + b * g.sA;
  const unsigned abytes = (unsigned)(g.lda * g.K * SZ);
  const unsigned bbytes = BK ? (unsigned)(g.bq * g.Q * SZ) : (unsigned)(g.bk * g.K * SZ);
  const __amdgpu_buffer_rsrc_t ra_src = make_rsrc(A, abytes);
  const __amdgpu_buffer_rsrc_t rb_src = make_rsrc(static_cast<const T*>(g.B), bbytes);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave % WGM) * WM, wq0 = (wave / WGM) * WQ;
  const int lr = lane & 15, lk = lane >> 4;

  // per-thread byte offsets of the chunk at k0 = 0
  unsigned va[AL], vb[BL];
#pragma unroll
  for (int p = 0; p < AL; ++p) {
    const int idx = tid + NT * p;
    const int m = idx % TM, k = idx / TM;
    va[p] = (m0 + m < Mi) ? ((unsigned)(m0 + m) + lda * (unsigned)k) * SZ : abytes;
  }
#pragma unroll
  for (int p = 0; p < BL; ++p) {
    const int idx = tid + NT * p;
    const int q = BK ? idx / KC : idx % TQ;
    const int k = BK ? idx % KC : idx / TQ;
    if (BK)  // k fastest: K validity is checked per chunk; a Q overrun leaves the tensor
      vb[p] = ((unsigned)k + bq * (unsigned)(q0 + q)) * SZ;
    else
      vb[p] = (q0 + q < Qi) ? ((unsigned)(q0 + q) + bk * (unsigned)k) * SZ : bbytes;
  }

  v4d acc[NP][FM][FQ];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FQ; ++j) acc[p][i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  auto gload = [&](T (&ra)[AL], T (&rb)[BL], int k0) {
    const unsigned sa = lda * (unsigned)k0 * SZ;
#pragma unroll
    for (int p = 0; p < AL; ++p) ra[p] = buffer_ld<T>(ra_src, va[p], sa);
    if constexpr (BK) {
#pragma unroll
      for (int p = 0; p < BL; ++p) {
        const int k = (tid + NT * p) % KC;
        rb[p] = buffer_ld<T>(rb_src, (k0 + k < Ki) ? vb[p] : bbytes, (unsigned)k0 * SZ);
      }
    } else {
      const unsigned sb = bk * (unsigned)k0 * SZ;
#pragma unroll
      for (int p = 0; p < BL; ++p) rb[p] = buffer_ld<T>(rb_src, vb[p], sb);
    }
  };
  // registers -> LDS buffer `buf` (complex data split into real and imaginary planes)
  auto sstore = [&](const T (&ra)[AL], const T (&rb)[BL], int buf) {
#pragma unroll
    for (int p = 0; p < AL; ++p) {
      const int idx = tid + NT * p;
      const int m = idx % TM, k = idx / TM;
      if constexpr (CPLX) {
        As(buf, 0, k * LDA_S + m) = ra[p].re;
        As(buf, 1, k * LDA_S + m) = ra[p].im;
      } else {
        As(buf, 0, k * LDA_S + m) = ra[p];
      }
    }
#pragma unroll
    for (int p = 0; p < BL; ++p) {
      const int idx = tid + NT * p;
      const int q = BK ? idx / KC : idx % TQ;
      const int k = BK ? idx % KC : idx / TQ;
      if constexpr (CPLX) {
        Bs(buf, 0, k * LDB_S + q) = rb[p].re;
        Bs(buf, 1, k * LDB_S + q) = rb[p].im;
      } else {
        Bs(buf, 0, k * LDB_S + q) = rb[p];
      }
    }
  };
  auto compute = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double af[NP][FM], bf[NP][FQ];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int i = 0; i < FM; ++i) af[p][i] = As(cur, p, (kk + lk) * LDA_S + wm0 + i * 16 + lr);
#pragma unroll
        for (int j = 0; j < FQ; ++j) bf[p][j] = Bs(cur, p, (kk + lk) * LDB_S + wq0 + j * 16 + lr);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FQ; ++j) {
          if constexpr (CPLX) {
            // (Ar + i Ai)(Br + i Bi) = (Ar Br - Ai Bi) + i (Ar Bi + Ai Br)
            acc[0][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[0][j], af[0][i], acc[0][i][j], 0, 0, 0);
            acc[0][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-bf[1][j], af[1][i], acc[0][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[0][j], af[1][i], acc[1][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[1][j], af[0][i], acc[1][i][j], 0, 0, 0);
          } else {
            acc[0][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[0][j], af[0][i], acc[0][i][j], 0, 0, 0);
          }
        }
    }
  };

  const int nk = (Ki + KC - 1) / KC;
  T ra[PF][AL], rb[PF][BL];
  if constexpr (PF == 2) {
    // Two register sets keep two K chunks in flight: while LDS buffer c is
    // consumed, chunk k+1 travels into the other register set and chunk k+2
    // is requested.  Loads inside the steady-state loop are unconditional (a
    // chunk past the end reads zeros from outside the buffer range without
    // touching memory), so the outstanding-load count is the same on every
    // path and each store waits only for its own chunk.  One barrier per
    // chunk; the tail (one or two chunks) is peeled.
    auto interleave = []() {
      if constexpr (IL) {
        constexpr int NM = NP * NP * FM * FQ * (KC / 4), NR = NP * (FM + FQ) * (KC / 4);
        constexpr int RPM = (NR + NM - 1) / NM, NW = NP * (AL + BL), NV = AL + BL;
#pragma unroll
        for (int u = 0; u < NM; ++u) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
          __builtin_amdgcn_sched_group_barrier(0x100, RPM, 0);  // LDS read
          if (u < NW) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
          if (u < NV) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // global load
        }
      }
    };
    gload(ra[0], rb[0], 0);
    gload(ra[1], rb[1], KC);
    sstore(ra[0], rb[0], 0);
    __syncthreads();
    int kc = 0;
    for (; kc + 2 < nk; kc += 2) {
      gload(ra[0], rb[0], (kc + 2) * KC);
      compute(0);
      sstore(ra[1], rb[1], 1);
      interleave();
      __syncthreads();
      gload(ra[1], rb[1], (kc + 3) * KC);
      compute(1);
      sstore(ra[0], rb[0], 0);
      interleave();
      __syncthreads();
    }
    compute(0);  // buffer 0 holds chunk kc, set 1 chunk kc + 1
    if (kc + 1 < nk) {
      sstore(ra[1], rb[1], 1);
      __syncthreads();
      compute(1);
    }
  } else {
    // PF register sets keep PF K chunks in flight.  At step c the LDS buffer
    // c mod 2 holds chunk c, the sets hold chunks c+1 .. c+PF-1, and the set
    // that held chunk c (already stored) requests chunk c+PF.
#pragma unroll
    for (int u = 0; u < PF; ++u) gload(ra[u], rb[u], u * KC);
    sstore(ra[0], rb[0], 0);
    __syncthreads();
    for (int kc = 0; kc < nk; kc += PF) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int c = kc + u;
        gload(ra[u], rb[u], (c + PF) * KC);
        if (c < nk) compute(c & 1);
        if (c + 1 < nk) sstore(ra[(u + 1) % PF], rb[(u + 1) % PF], (c + 1) & 1);
        __syncthreads();
      }
    }
  }

  // acc[.][i][j][r] holds C[m, q] with m = wm0 + 16 i + (lane mod 16),
  // q = wq0 + 16 j + (lane / 16) + 4 r
  const long cbase = b * g.sC;
  epilogue_tile<T>(g.epi, [&](auto&& f) {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int m = m0 + wm0 + i * 16 + lr;
      if (m >= Mi) continue;
#pragma unroll
      for (int j = 0; j < FQ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + wq0 + j * 16 + lk + 4 * r;
          if (q >= Qi) continue;
          const long e = cbase + m + g.ldc * (long)q;
          if constexpr (CPLX)
            f(e, cdouble{acc[0][i][j][r], acc[1][i][j][r]});
          else
            f(e, acc[0][i][j][r]);
        }
    }
  });
}

template <typename T, bool BK, int TM, int TQ, int KC, int WGM, int WGQ, int PF, bool IL>
__global__ __launch_bounds__(64 * WGM * WGQ) void k_mode_product(GemmArgs g) {
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  gemm_tile<T, BK, TM, TQ, KC, WGM, WGQ, PF, tile_lds_doubles<T, BK, TM, TQ, KC>(), IL>(
      g, xcd_remap((long)blockIdx.x, nt));
}

// Tile classes of the grouped launch: TM x TQ outputs, K chunks of KC, WGM x WGQ
// waves (both classes of a launch on the same thread count), registers for WPE
// waves per SIMD.
template <int TM_, int TQ_, int KC_, int WGM_, int WGQ_, int WPE_ = 4, bool IL_ = false>
struct TileCfg {
  static constexpr int TM = TM_, TQ = TQ_, KC = KC_, WGM = WGM_, WGQ = WGQ_, NT = 64 * WGM_ * WGQ_;
  static constexpr int WPE = WPE_;  // waves per SIMD the kernel's registers must allow
  static constexpr bool IL = IL_;   // interleaved chunk schedule (gemm_tile)
};
using GSmall = TileCfg<64, 64, 32, 2, 4>;
using GSmall4 = TileCfg<64, 64, 16, 2, 2>;
using GSmall16 = TileCfg<64, 64, 16, 2, 4, 6>;
using GSmall16x = TileCfg<64, 64, 16, 2, 4, 8>;
using GBig = TileCfg<128, 64, 16, 4, 2>;
using GBig8 = TileCfg<128, 64, 8, 4, 2, 6>;

// Grouped GEMM: independent GEMMs (one descriptor each, tile class and tile
// counts filled in) share one launch.  Workgroup b runs tile map[b].tile of
// descriptor map[b].desc (none if desc < 0); the host builds the map so that
// each GEMM's tiles run on one XCD (grouped_block_map).  A descriptor of class
// 1 runs on L tiles, class 0 on S tiles; both use one LDS allocation (the
// larger of the two).
template <bool BK, class S, class L>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(S::WPE))) void k_grouped_gemm(
    const GemmArgs* __restrict__ descs, const GroupedBlock* __restrict__ map) {
  constexpr int LS = tile_lds_doubles<double, BK, S::TM, S::TQ, S::KC>();
  constexpr int LL = tile_lds_doubles<double, BK, L::TM, L::TQ, L::KC>();
  constexpr int LN = LS > LL ? LS : LL;
  static_assert(S::NT == L::NT, "both tile classes run on the same waves");
  const GroupedBlock e = map[blockIdx.x];
  if (e.desc < 0) return;
  const GemmArgs g = descs[e.desc];
  if (g.gate && *g.gate <= g.gate_level) return;  // uniform over the workgroup
  if constexpr (std::is_same<S, L>::value) {
    gemm_tile<double, BK, S::TM, S::TQ, S::KC, S::WGM, S::WGQ, 2, LN, S::IL>(g, e.tile);
  } else {
    if (g.cls)
      gemm_tile<double, BK, L::TM, L::TQ, L::KC, L::WGM, L::WGQ, 2, LN, L::IL>(g, e.tile);
    else
      gemm_tile<double, BK, S::TM, S::TQ, S::KC, S::WGM, S::WGQ, 2, LN, S::IL>(g, e.tile);
  }
}

template <typename T, bool BK, int TM, int TQ, int KC, int WGM, int WGQ, int PF = 2, bool IL = false>
int launch_tile(GemmArgs& g, hipStream_t s) {
  set_tile_counts(g, TM, TQ);
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  if (nt <= 0) return EXPINT_OK;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "mode product: too many tiles (%ld)", nt);
  hipLaunchKernelGGL((k_mode_product<T, BK, TM, TQ, KC, WGM, WGQ, PF, IL>), dim3((unsigned)nt), dim3(64 * WGM * WGQ),
                     0, s, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "mode product launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

// Tile configurations (TM x TQ outputs per workgroup; "w8" = 8 waves, else 4;
// "k32" K chunks of 32; "p3" / "p4" that many register sets in flight; "i" the
// interleaved chunk schedule).  EXPINT_TILE set to one of these names overrides
// the automatic choice.
const char* const kTileNames[] = {"64x64", "64x32", "32x64", "128x64", "64x128", "32x32",
                                  "64x64w8", "128x64w8", "128x128w8", "128x128", "128x64w8k32", "128x128w8k32",
                                  "128x64w8p3", "128x64w8p4", "64x64w8p3", "64x64w8p4", "64x64k32", "128x64w8i",
                                  "64x64w8i"};
constexpr int kNumTiles = sizeof(kTileNames) / sizeof(kTileNames[0]);

// Measured on MI355X (FP64, K = n): 128x64 outputs on 8 waves is the fastest
// real tile from 128^3 to 384^3 (69% of the FP64 MFMA peak at 384^3); complex
// data, with four MFMAs per output block, does best on 64x64 / 8 waves.
// Narrow M (short contiguous dimension) takes 32-row tiles to waste less.
// Measured choice (MI355X sweep over the table above).  Real data: 128 x 64
// on 8 waves, unless that leaves fewer than two tiles per CU (256 CUs); then
// 64 x 64 on 4 waves, whose twice as many workgroups overlap each other's
// prologue and store burst (128^3: 15.2 instead of 15.8 us per launch).
// The autotuner's choice (or EXPINT_TILE) comes first.
int choose_tile(bool cplx, long M, long Q, long K, long batches) {
  const int o = tune_choice(TuneKey{cplx ? TUNE_MP_CPLX : TUNE_MP_REAL, M, Q, K, batches});
  if (o >= 0) return o;
  if (cplx) return M >= 64 ? 6 : 2;
  if (M >= 128) {
    const long big = ((M + 127) / 128) * ((Q + 63) / 64) * batches;
    return big < 512 ? 0 : 7;
  }
  if (M >= 64) return 6;
  return 2;
}

template <typename T, bool BK>
int launch_choice(GemmArgs& g, hipStream_t st) {
  constexpr int KCR = std::is_same<T, cdouble>::value ? 8 : 16;
  switch (choose_tile(std::is_same<T, cdouble>::value, g.M, g.Q, g.K, g.batches)) {
    case 1: return launch_tile<T, BK, 64, 32, KCR, 2, 2>(g, st);
    case 2: return launch_tile<T, BK, 32, 64, KCR, 2, 2>(g, st);
    case 3: return launch_tile<T, BK, 128, 64, KCR, 2, 2>(g, st);
    case 4: return launch_tile<T, BK, 64, 128, KCR, 2, 2>(g, st);
    case 5: return launch_tile<T, BK, 32, 32, KCR * 2, 2, 2>(g, st);
    case 6: return launch_tile<T, BK, 64, 64, KCR * 2, 2, 4>(g, st);
    case 7: return launch_tile<T, BK, 128, 64, KCR, 4, 2>(g, st);
    case 8: return launch_tile<T, BK, 128, 128, KCR, 4, 2>(g, st);
    case 9: return launch_tile<T, BK, 128, 128, KCR, 2, 2>(g, st);
    case 10: return launch_tile<T, BK, 128, 64, KCR * 2, 4, 2>(g, st);
    case 11: return launch_tile<T, BK, 128, 128, KCR * 2, 4, 2>(g, st);
    case 12: return launch_tile<T, BK, 128, 64, KCR, 4, 2, 3>(g, st);
    case 13: return launch_tile<T, BK, 128, 64, KCR, 4, 2, 4>(g, st);
    case 14: return launch_tile<T, BK, 64, 64, KCR * 2, 2, 4, 3>(g, st);
    case 15: return launch_tile<T, BK, 64, 64, KCR * 2, 2, 4, 4>(g, st);
    case 16: return launch_tile<T, BK, 64, 64, KCR * 2, 2, 2>(g, st);
    case 17: return launch_tile<T, BK, 128, 64, KCR, 4, 2, 2, true>(g, st);
    case 18: return launch_tile<T, BK, 64, 64, KCR * 2, 2, 4, 2, true>(g, st);
    default: return launch_tile<T, BK, 64, 64, KCR, 2, 2>(g, st);
  }
}

}  // namespace

int mode_product_tile_count() { return kNumTiles; }
const char* mode_product_tile_name(int i) { return i >= 0 && i < kNumTiles ? kTileNames[i] : "?"; }

// the GEMM launch_mode_product makes: mode 1 (s == 1) is M = n, Q = r, one batch;
// modes >= 2 are M = s, Q = n, r batches; K = n either way
TuneKey mode_product_key(bool cplx, long s, int n, long r) {
  if (s == 1) return TuneKey{cplx ? TUNE_MP_CPLX : TUNE_MP_REAL, n, r, n, 1};
  return TuneKey{cplx ? TUNE_MP_CPLX : TUNE_MP_REAL, s, n, n, r};
}

// Grouped tile schemes: which tile class each GEMM of a grouped launch takes,
// and the tile shapes (outputs TM x TQ, K chunk KC, waves, workgroups per CU).
//   "64x64k16"           every GEMM on 64 x 64 tiles, K chunks of 16, 8 waves, 3 per CU (default)
//   "64x64k16o4"         the same with registers for 4 workgroups per CU
//   "64x64"              64 x 64 tiles, K chunks of 32, 8 waves, 2 per CU
//   "64x64w4"            64 x 64 tiles, K chunks of 16, 4 waves, 4 per CU
//   "128x64"             every GEMM on 128 x 64 tiles, K chunks of 16, 8 waves, 2 per CU
//   "128x64k8"           128 x 64 tiles, K chunks of 8, 8 waves, 3 per CU
//   "64x64+128x64"       GEMMs with M >= 128 on 128 x 64 tiles, the rest 64 x 64 (K chunks 16 / 32)
//   "64x64k16+128x64k8"  GEMMs with M >= 128 on 128 x 64 tiles (K chunks of 8), the rest 64 x 64 (16)
// The two-class schemes serve both classes from one launch and one LDS
// allocation.  EXPINT_GROUPED set to one of these names overrides the tuned choice.
// Each tile scheme comes with two workgroup maps (grouped_block_map): balanced by
// multiply-adds (the name alone) or with a per-tile allowance for the prologue and
// epilogue and finer runs (the name with ",lpt64").
const char* const kGroupedNames[] = {"64x64k16",           "64x64k16o4",           "64x64",
                                     "64x64w4",            "128x64",               "128x64k8",
                                     "64x64+128x64",       "64x64k16+128x64k8",    "64x64k16,lpt64",
                                     "64x64k16o4,lpt64",   "64x64,lpt64",          "64x64w4,lpt64",
                                     "128x64,lpt64",       "128x64k8,lpt64",       "64x64+128x64,lpt64",
                                     "64x64k16+128x64k8,lpt64"};
constexpr int kNumGrouped = sizeof(kGroupedNames) / sizeof(kGroupedNames[0]);
constexpr int kNumTileSchemes = kNumGrouped / 2;

int grouped_scheme_count() { return kNumGrouped; }
const char* grouped_scheme_name(int i) { return i >= 0 && i < kNumGrouped ? kGroupedNames[i] : "?"; }

// the class (0 small, 1 large) and tile shape of an M x Q GEMM under a scheme
static int grouped_class(int scheme, long M, long Q, int* tm, int* tq) {
  (void)Q;
  int cls = 0;
  switch (scheme % kNumTileSchemes) {
    case 4:
    case 5: cls = 1; break;
    case 6:
    case 7: cls = M >= 128; break;
    default: cls = 0;
  }
  *tm = cls ? 128 : 64;
  *tq = 64;
  return cls;
}

void gemm_desc_set_scheme(void* desc, int scheme) {
  GemmArgs g;
  std::memcpy(&g, desc, sizeof(g));
  int tm, tq;
  g.cls = grouped_class(scheme, g.M, g.Q, &tm, &tq);
  g.tile_m = tm;
  g.tile_q = tq;
  set_tile_counts(g, tm, tq);
  std::memcpy(desc, &g, sizeof(g));
}

template <bool BK, class S, class L>
static void launch_grouped_typed(long grid, const GemmArgs* d, const GroupedBlock* map, hipStream_t st) {
  hipLaunchKernelGGL((k_grouped_gemm<BK, S, L>), dim3((unsigned)grid), dim3(S::NT), 0, st, d, map);
}

template <bool BK>
static void launch_grouped_scheme(int scheme, long grid, const GemmArgs* d, const GroupedBlock* map, hipStream_t st) {
  switch (scheme % kNumTileSchemes) {
    case 1: return launch_grouped_typed<BK, GSmall16x, GSmall16x>(grid, d, map, st);
    case 2: return launch_grouped_typed<BK, GSmall, GSmall>(grid, d, map, st);
    case 3: return launch_grouped_typed<BK, GSmall4, GSmall4>(grid, d, map, st);
    case 4: return launch_grouped_typed<BK, GBig, GBig>(grid, d, map, st);
    case 5: return launch_grouped_typed<BK, GBig8, GBig8>(grid, d, map, st);
    case 6: return launch_grouped_typed<BK, GSmall, GBig>(grid, d, map, st);
    case 7: return launch_grouped_typed<BK, GSmall16, GBig8>(grid, d, map, st);
    default: return launch_grouped_typed<BK, GSmall16, GSmall16>(grid, d, map, st);
  }
}

int launch_grouped_gemm(bool bk_contiguous, const void* descs, const GroupedBlock* map, long blocks, int scheme,
                        void* stream) {
  if (blocks <= 0) return EXPINT_OK;
  if (blocks > 0x7fffffffL) return set_error(EXPINT_EINVAL, "grouped GEMM: too many workgroups (%ld)", blocks);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const GemmArgs* d = static_cast<const GemmArgs*>(descs);
  if (bk_contiguous)
    launch_grouped_scheme<true>(scheme, blocks, d, map, st);
  else
    launch_grouped_scheme<false>(scheme, blocks, d, map, st);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "grouped GEMM launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

size_t gemm_desc_size() { return sizeof(GemmArgs); }

int make_gemm_desc(void* out, const void* A, long lda, const void* B, long bk, long bq, long M, long Q, long K,
                   long ldc, const Epilogue& epi, const int* gate, int gate_level) {
  GemmArgs g;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.bk = bk;
  g.bq = bq;
  g.M = M;
  g.Q = Q;
  g.K = K;
  g.sA = 0;
  g.sC = 0;
  g.ldc = ldc;
  g.batches = 1;
  g.epi = epi;
  g.gate = gate;
  g.gate_level = gate_level;
  int tm, tq;
  g.cls = grouped_class(0, M, Q, &tm, &tq);
  g.tile_m = tm;
  g.tile_q = tq;
  set_tile_counts(g, tm, tq);
  std::memcpy(out, &g, sizeof(g));
  return EXPINT_OK;
}

// The workgroup -> tile map of a grouped launch.  Workgroups are dispatched to
// the XCDs in turn (b mod 8), and each XCD has its own L2, so the tiles of one
// GEMM, which re-read each other's operand panels, are kept on one XCD: the
// GEMMs (split into runs of at most an eighth of all tiles, so that no XCD
// holds much more than its share) go to the XCDs longest first, each to the
// XCD with the least work so far (work = tiles x TM TQ K); within an XCD the
// runs keep that order.  The ",lpt64" schemes add 64 to K for each tile's
// prologue and epilogue and cut runs at a sixteenth (measured on the
// 64-instance batch: ETD2RK 0.71 ms per step with the first measure against
// 0.74 with the second, Rosenbrock-Euler the other way round, 7.36 against
// 7.53).  XCD x's j-th tile becomes workgroup 8 j + x; a workgroup past the end
// of its XCD's list has desc = -1.  EXPINT_GROUPED_FLAT=1 gives the plain order
// (tile t on workgroup t) instead.
void grouped_block_map(const void* descs, int count, int scheme, std::vector<GroupedBlock>& map) {
  constexpr int X = 8;
  const GemmArgs* d = static_cast<const GemmArgs*>(descs);
  std::vector<long> tiles(count);
  long total = 0;
  for (int i = 0; i < count; ++i) {
    GemmArgs g;
    std::memcpy(&g, d + i, sizeof(g));
    tiles[i] = g.tiles_m * g.tiles_q * g.batches;
    total += tiles[i];
  }
  map.clear();
  if (const char* e = std::getenv("EXPINT_GROUPED_FLAT"); e && std::strcmp(e, "1") == 0) {
    for (int i = 0; i < count; ++i)
      for (long t = 0; t < tiles[i]; ++t) map.push_back(GroupedBlock{i, (int)t});
    return;
  }
  struct Run {
    int desc;
    long t0, t1;
    double work;
  };
  const bool lpt64 = scheme >= kNumTileSchemes;
  const long cap = lpt64 ? std::max(1L, (total + 15) / 16) : std::max(1L, (total + 7) / 8);
  std::vector<Run> runs;
  for (int i = 0; i < count; ++i) {
    GemmArgs g;
    std::memcpy(&g, d + i, sizeof(g));
    const double per = (double)g.tile_m * g.tile_q * (double)(g.K + (lpt64 ? 64 : 0));
    for (long t0 = 0; t0 < tiles[i]; t0 += cap) {
      const long t1 = std::min(tiles[i], t0 + cap);
      runs.push_back(Run{i, t0, t1, per * (double)(t1 - t0)});
    }
  }
  std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.work > b.work; });
  std::vector<std::vector<GroupedBlock>> lists(X);
  double load[X] = {0};
  for (const Run& r : runs) {
    int x = 0;
    for (int k = 1; k < X; ++k)
      if (load[k] < load[x]) x = k;
    load[x] += r.work;
    for (long t = r.t0; t < r.t1; ++t) lists[x].push_back(GroupedBlock{r.desc, (int)t});
  }
  size_t longest = 0;
  for (const auto& l : lists) longest = std::max(longest, l.size());
  map.assign(longest * X, GroupedBlock{-1, 0});
  for (int x = 0; x < X; ++x)
    for (size_t j = 0; j < lists[x].size(); ++j) map[j * X + x] = lists[x][j];
}

// Every tile of every descriptor exactly once, nothing out of range.
bool grouped_block_map_valid(const void* descs, int count, const std::vector<GroupedBlock>& map) {
  const GemmArgs* d = static_cast<const GemmArgs*>(descs);
  std::vector<long> base(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    GemmArgs g;
    std::memcpy(&g, d + i, sizeof(g));
    base[i + 1] = base[i] + g.tiles_m * g.tiles_q * g.batches;
  }
  std::vector<char> seen(base[count], 0);
  for (const GroupedBlock& e : map) {
    if (e.desc < 0) continue;
    if (e.desc >= count || e.tile < 0 || e.tile >= base[e.desc + 1] - base[e.desc]) return false;
    char& f = seen[base[e.desc] + e.tile];
    if (f) return false;
    f = 1;
  }
  for (char f : seen)
    if (!f) return false;
  return true;
}

long gemm_desc_tiles(const void* desc) {
  GemmArgs g;
  std::memcpy(&g, desc, sizeof(g));
  return g.tiles_m * g.tiles_q * g.batches;
}

int launch_mode_product(int dtype, long s, int n, long r, const void* M, const void* V,
                        const Epilogue& epi, void* stream) {
  if (s <= 0 || n <= 0 || r <= 0) return EXPINT_OK;
  // buffer-resource offsets are 32-bit; with operands below 2 GiB an operand's
  // range plus its largest K offset still fits
  const long bytes = s * (long)n * r * (dtype == EXPINT_C128 ? 16 : 8);
  if (bytes >= (1L << 31))
    return set_error(EXPINT_ENOTSUP, "mode product: tensors of %ld bytes exceed the 2 GiB limit", bytes);
  GemmArgs g;
  g.epi = epi;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool cplx = dtype == EXPINT_C128;
  if (s == 1) {
    // C[i, c] = sum_j M[i, j] V[j, c]; Aop = M, Bop = V (k fastest)
    g.A = M;
    g.lda = n;
    g.B = V;
    g.bk = 1;
    g.bq = n;
    g.M = n;
    g.Q = r;
    g.K = n;
    g.sA = 0;
    g.sC = 0;
    g.ldc = n;
    g.batches = 1;
    return cplx ? launch_choice<cdouble, true>(g, st) : launch_choice<double, true>(g, st);
  }
  // per outer index b: C[a, i] = sum_j V[a, j, b] M[i, j]; Aop = V slab, Bop = M^T
  g.A = V;
  g.lda = s;
  g.B = M;
  g.bk = n;
  g.bq = 1;
  g.M = s;
  g.Q = n;
  g.K = n;
  g.sA = s * (long)n;
  g.sC = s * (long)n;
  g.ldc = s;
  g.batches = r;
  return cplx ? launch_choice<cdouble, false>(g, st) : launch_choice<double, false>(g, st);
}

}  // namespace expint

// ===========================================================================
// Reduced-precision contractions of the same mu-mode product.
//
// The phi matrices and the state stay FP64; only the contraction is done in
// lower precision (the paper names single and half precision as future work
// for GPU runs, section 5).  Two variants, both with FP32 accumulation:
//   FP32    operands rounded to FP32, v_mfma_f32_16x16x4f32;
//   BF16X3  x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
//           even), x*y ~ hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16.
// Inner modes write FP32 intermediates; the last mode converts its FP32
// result to FP64 and runs the FP64 epilogue.  For both MFMAs D[i][j] sits in
// lane j + 16 (i / 4), register i mod 4 (probed on the device), so with the
// B fragment as first operand the 16 lanes of a row group hold 16
// consecutive outputs m.
// ===========================================================================
namespace expint {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct __attribute__((aligned(8))) cfloat {
  float re, im;
};
template <typename T> struct is_cplx : std::false_type {};
template <> struct is_cplx<cdouble> : std::true_type {};
template <> struct is_cplx<cfloat> : std::true_type {};
__device__ __forceinline__ float re_f(double x) { return (float)x; }
__device__ __forceinline__ float re_f(float x) { return x; }
__device__ __forceinline__ float re_f(cdouble x) { return (float)x.re; }
__device__ __forceinline__ float re_f(cfloat x) { return x.re; }
__device__ __forceinline__ float im_f(cdouble x) { return (float)x.im; }
__device__ __forceinline__ float im_f(cfloat x) { return x.im; }
template <typename T> __device__ __forceinline__ float im_f(T) { return 0.f; }

template <typename T>
__device__ __forceinline__ T buffer_ld_s(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ double buffer_ld_s<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ float buffer_ld_s<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ cdouble buffer_ld_s<cdouble>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cdouble, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ cfloat buffer_ld_s<cfloat>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(cfloat, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

struct GemmArgsLP {
  GemmArgs g;      // shapes, strides, epilogue (out0 is float* when out32)
};

// Stores of the reduced-precision kernels: an FP32 intermediate tensor is
// written as it is, the last mode goes through the FP64 epilogue.
template <bool OUT32, bool CPLX, typename Elems>
__device__ __forceinline__ void lp_store_tile(const Epilogue& ep, Elems&& elems) {
  if constexpr (OUT32) {
    if constexpr (CPLX)
      elems([&](long e, float yr, float yi) { static_cast<cfloat*>(ep.out0)[e] = cfloat{yr, yi}; });
    else
      elems([&](long e, float y, float) { static_cast<float*>(ep.out0)[e] = y; });
  } else if constexpr (CPLX) {
    epilogue_tile<cdouble>(ep, [&](auto&& f) {
      elems([&](long e, float yr, float yi) { f(e, cdouble{(double)yr, (double)yi}); });
    });
  } else {
    epilogue_tile<double>(ep, [&](auto&& f) { elems([&](long e, float y, float) { f(e, (double)y); }); });
  }
}

// ---------------------------------------------------------------------------
// FP32: structure of the FP64 kernel with an FP32 LDS and f32 MFMA
// ---------------------------------------------------------------------------
template <typename TA, typename TB, bool OUT32, bool BK, int TM, int TQ, int KC, int WGM, int WGQ>
__global__ __launch_bounds__(64 * WGM * WGQ) void k_mode_product_f32(GemmArgs g) {
  constexpr bool CPLX = is_cplx<TA>::value;
  static_assert(CPLX == is_cplx<TB>::value, "operands must both be real or both complex");
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int NT = 64 * WGM * WGQ;
  constexpr unsigned SA = sizeof(TA), SB = sizeof(TB);
  constexpr int LDA_S = TM, LDB_S = BK ? TQ + 1 : TQ;
  constexpr int WM = TM / WGM, WQ = TQ / WGQ;
  constexpr int FM = WM / 16, FQ = WQ / 16;
  constexpr int AL = TM * KC / NT, BL = TQ * KC / NT;
  static_assert(AL * NT == TM * KC && BL * NT == TQ * KC, "tile / thread mismatch");
  static_assert(FM >= 1 && FQ >= 1 && KC % 4 == 0, "bad tile");
  __shared__ float As[2][NP][KC * LDA_S];
  __shared__ float Bs[2][NP][KC * LDB_S];

  const long nt = g.tiles_m * g.tiles_q * g.batches;
  const long T_ = xcd_remap((long)blockIdx.x, nt);
  const TileCoord tc = tile_coord(T_, g.tiles_m, g.tiles_q, g.m_fastest);
  const long tm = tc.tm, tq = tc.tq, b = tc.b;
  const int m0 = (int)(tm * TM), q0 = (int)(tq * TQ);
  const int Mi = (int)g.M, Qi = (int)g.Q, Ki = (int)g.K;
  const unsigned lda = (unsigned)g.lda, bk = (unsigned)g.bk, bq = (unsigned)g.bq;
  const TA* A = static_cast<const TA*>(g.A) + b * g.sA;
  const unsigned abytes = (unsigned)(g.lda * g.K * SA);
  const unsigned bbytes = BK ? (unsigned)(g.bq * g.Q * SB) : (unsigned)(g.bk * g.K * SB);
  const __amdgpu_buffer_rsrc_t ra_src = make_rsrc(A, abytes);
  const __amdgpu_buffer_rsrc_t rb_src = make_rsrc(static_cast<const TB*>(g.B), bbytes);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % WGM) * WM, wq0 = (wave / WGM) * WQ;
  const int lr = lane & 15, lk = lane >> 4;

  unsigned va[AL], vb[BL];
#pragma unroll
  for (int p = 0; p < AL; ++p) {
    const int idx = tid + NT * p, m = idx % TM, k = idx / TM;
    va[p] = (m0 + m < Mi) ? ((unsigned)(m0 + m) + lda * (unsigned)k) * SA : abytes;
  }
#pragma unroll
  for (int p = 0; p < BL; ++p) {
    const int idx = tid + NT * p;
    const int q = BK ? idx / KC : idx % TQ, k = BK ? idx % KC : idx / TQ;
    if (BK)
      vb[p] = ((unsigned)k + bq * (unsigned)(q0 + q)) * SB;
    else
      vb[p] = (q0 + q < Qi) ? ((unsigned)(q0 + q) + bk * (unsigned)k) * SB : bbytes;
  }
  v4f acc[NP][FM][FQ];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FQ; ++j) acc[p][i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto gload = [&](TA (&ra)[AL], TB (&rb)[BL], int k0) {
    const unsigned sa = lda * (unsigned)k0 * SA;
#pragma unroll
    for (int p = 0; p < AL; ++p) ra[p] = buffer_ld_s<TA>(ra_src, va[p], sa);
    if constexpr (BK) {
#pragma unroll
      for (int p = 0; p < BL; ++p) {
        const int k = (tid + NT * p) % KC;
        rb[p] = buffer_ld_s<TB>(rb_src, (k0 + k < Ki) ? vb[p] : bbytes, (unsigned)k0 * SB);
      }
    } else {
      const unsigned sb = bk * (unsigned)k0 * SB;
#pragma unroll
      for (int p = 0; p < BL; ++p) rb[p] = buffer_ld_s<TB>(rb_src, vb[p], sb);
    }
  };
  auto sstore = [&](const TA (&ra)[AL], const TB (&rb)[BL], int buf) {
#pragma unroll
    for (int p = 0; p < AL; ++p) {
      const int idx = tid + NT * p, m = idx % TM, k = idx / TM;
      As[buf][0][k * LDA_S + m] = re_f(ra[p]);
      if constexpr (CPLX) As[buf][1][k * LDA_S + m] = im_f(ra[p]);
    }
#pragma unroll
    for (int p = 0; p < BL; ++p) {
      const int idx = tid + NT * p;
      const int q = BK ? idx / KC : idx % TQ, k = BK ? idx % KC : idx / TQ;
      Bs[buf][0][k * LDB_S + q] = re_f(rb[p]);
      if constexpr (CPLX) Bs[buf][1][k * LDB_S + q] = im_f(rb[p]);
    }
  };
  auto compute = [&](int cur) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      float af[NP][FM], bf[NP][FQ];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int i = 0; i < FM; ++i) af[p][i] = As[cur][p][(kk + lk) * LDA_S + wm0 + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < FQ; ++j) bf[p][j] = Bs[cur][p][(kk + lk) * LDB_S + wq0 + j * 16 + lr];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FQ; ++j) {
          if constexpr (CPLX) {
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[0][j], af[0][i], acc[0][i][j], 0, 0, 0);
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-bf[1][j], af[1][i], acc[0][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[0][j], af[1][i], acc[1][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[1][j], af[0][i], acc[1][i][j], 0, 0, 0);
          } else {
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[0][j], af[0][i], acc[0][i][j], 0, 0, 0);
          }
        }
    }
  };
  const int nk = (Ki + KC - 1) / KC;
  TA ra0[AL], ra1[AL];
  TB rb0[BL], rb1[BL];
  gload(ra0, rb0, 0);
  gload(ra1, rb1, KC);
  sstore(ra0, rb0, 0);
  __syncthreads();
  int kc = 0;
  for (; kc + 2 < nk; kc += 2) {
    gload(ra0, rb0, (kc + 2) * KC);
    compute(0);
    sstore(ra1, rb1, 1);
    __syncthreads();
    gload(ra1, rb1, (kc + 3) * KC);
    compute(1);
    sstore(ra0, rb0, 0);
    __syncthreads();
  }
  compute(0);
  if (kc + 1 < nk) {
    sstore(ra1, rb1, 1);
    __syncthreads();
    compute(1);
  }
  // acc[i][j][r]: m = wm0 + 16 i + (lane mod 16), q = wq0 + 16 j + 4 (lane / 16) + r
  const long cbase = b * g.sC;
  lp_store_tile<OUT32, CPLX>(g.epi, [&](auto&& f) {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int m = m0 + wm0 + i * 16 + lr;
      if (m >= Mi) continue;
#pragma unroll
      for (int j = 0; j < FQ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + wq0 + j * 16 + 4 * lk + r;
          if (q >= Qi) continue;
          f(cbase + m + g.ldc * (long)q, acc[0][i][j][r], CPLX ? acc[NP - 1][i][j][r] : 0.0f);
        }
    }
  });
}

// ---------------------------------------------------------------------------
// BF16X3: K-major LDS (each lane reads its 8 consecutive k with one 16-byte
// LDS load), operands split into hi/lo planes when the chunk is stored.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;                 // round to nearest even
  lo = (__bf16)(x - (float)hi);   // exact difference in FP32, rounded to nearest even
}

// BV (with BK): a column of Bop starts on a 16-byte boundary, so each thread's
// 8 consecutive K values load as 16-byte vectors (values past K are zeroed).
template <typename TA, typename TB, bool OUT32, bool BK, int TM, int TQ, int WGM, int WGQ, bool BV = false>
__global__ __launch_bounds__(64 * WGM * WGQ) void k_mode_product_bf16x3(GemmArgs g) {
  constexpr int NT = 64 * WGM * WGQ;
  constexpr int KC = 32;                   // one MFMA K step per chunk
  constexpr int LDK = KC + 8;              // padded K-major row (bf16 elements)
  constexpr unsigned SA = sizeof(TA), SB = sizeof(TB);
  constexpr int WM = TM / WGM, WQ = TQ / WGQ;
  constexpr int FM = WM / 16, FQ = WQ / 16;
  constexpr int AG = TM * KC / 8 / NT, BG = TQ * KC / 8 / NT;   // 8-element groups per thread
  static_assert(AG * NT * 8 == TM * KC && BG * NT * 8 == TQ * KC, "tile / thread mismatch");
  static_assert(FM >= 1 && FQ >= 1, "bad tile");
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][TM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][TM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][TQ * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][TQ * LDK];

  const long nt = g.tiles_m * g.tiles_q * g.batches;
  const long T_ = xcd_remap((long)blockIdx.x, nt);
  const TileCoord tc = tile_coord(T_, g.tiles_m, g.tiles_q, g.m_fastest);
  const long tm = tc.tm, tq = tc.tq, b = tc.b;
  const int m0 = (int)(tm * TM), q0 = (int)(tq * TQ);
  const int Mi = (int)g.M, Qi = (int)g.Q, Ki = (int)g.K;
  const unsigned lda = (unsigned)g.lda, bk = (unsigned)g.bk, bq = (unsigned)g.bq;
  const TA* A = static_cast<const TA*>(g.A) + b * g.sA;
  const unsigned abytes = (unsigned)(g.lda * g.K * SA);
  const unsigned bbytes = BK ? (unsigned)(g.bq * g.Q * SB) : (unsigned)(g.bk * g.K * SB);
  const __amdgpu_buffer_rsrc_t ra_src = make_rsrc(A, abytes);
  const __amdgpu_buffer_rsrc_t rb_src = make_rsrc(static_cast<const TB*>(g.B), bbytes);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % WGM) * WM, wq0 = (wave / WGM) * WQ;
  const int lr = lane & 15, lk = lane >> 4;

  // group p of this thread: A covers (m, 8 kg .. 8 kg + 7) with m fastest over threads;
  // B likewise with q fastest, or (BK) 8 consecutive k of one column with kg fastest.
  unsigned va[AG], vb[BG];
#pragma unroll
  for (int p = 0; p < AG; ++p) {
    const int gi = tid + NT * p, m = gi % TM, kg = gi / TM;
    va[p] = (m0 + m < Mi) ? ((unsigned)(m0 + m) + lda * (unsigned)(8 * kg)) * SA : abytes;
  }
#pragma unroll
  for (int p = 0; p < BG; ++p) {
    const int gi = tid + NT * p;
    if (BK) {
      const int kg = gi % (KC / 8), q = gi / (KC / 8);
      vb[p] = ((unsigned)(8 * kg) + bq * (unsigned)(q0 + q)) * SB;
    } else {
      const int q = gi % TQ, kg = gi / TQ;
      vb[p] = (q0 + q < Qi) ? ((unsigned)(q0 + q) + bk * (unsigned)(8 * kg)) * SB : bbytes;
    }
  }
  v4f acc[FM][FQ];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FQ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  auto gload = [&](TA (&ra)[AG][8], TB (&rb)[BG][8], int k0) {
#pragma unroll
    for (int p = 0; p < AG; ++p)
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[p][e] = buffer_ld_s<TA>(ra_src, va[p], lda * (unsigned)(k0 + e) * SA);
#pragma unroll
    for (int p = 0; p < BG; ++p) {
      if constexpr (BK && BV) {
        const int kg = (tid + NT * p) % (KC / 8);
        constexpr int PER = 16 / SB;  // elements per 16-byte load
#pragma unroll
        for (int v = 0; v < 8 / PER; ++v) {
          const v4i w = __builtin_bit_cast(
              v4i, __builtin_amdgcn_raw_buffer_load_b128(rb_src, (int)(vb[p] + 16u * v), (int)(k0 * SB), 0));
#pragma unroll
          for (int e = 0; e < PER; ++e) {
            TB x;
            if constexpr (SB == 4)
              x = __builtin_bit_cast(float, w[e]);
            else
              x = __builtin_bit_cast(double, (unsigned long long)(unsigned)w[2 * e] |
                                                 ((unsigned long long)(unsigned)w[2 * e + 1] << 32));
            rb[p][PER * v + e] = (k0 + 8 * kg + PER * v + e < Ki) ? x : TB(0);
          }
        }
      } else if constexpr (BK) {
        const int kg = (tid + NT * p) % (KC / 8);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          rb[p][e] = buffer_ld_s<TB>(rb_src, (k0 + 8 * kg + e < Ki) ? vb[p] + (unsigned)e * SB : bbytes,
                                     (unsigned)k0 * SB);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) rb[p][e] = buffer_ld_s<TB>(rb_src, vb[p], bk * (unsigned)(k0 + e) * SB);
      }
    }
  };
  auto sstore = [&](const TA (&ra)[AG][8], const TB (&rb)[BG][8], int buf) {
#pragma unroll
    for (int p = 0; p < AG; ++p) {
      const int gi = tid + NT * p, m = gi % TM, kg = gi / TM;
      v8bf hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 h, l;
        split_bf16((float)ra[p][e], h, l);
        hi[e] = h;
        lo[e] = l;
      }
      *reinterpret_cast<v8bf*>(&Ah[buf][m * LDK + 8 * kg]) = hi;
      *reinterpret_cast<v8bf*>(&Al[buf][m * LDK + 8 * kg]) = lo;
    }
#pragma unroll
    for (int p = 0; p < BG; ++p) {
      const int gi = tid + NT * p;
      const int q = BK ? gi / (KC / 8) : gi % TQ;
      const int kg = BK ? gi % (KC / 8) : gi / TQ;
      v8bf hi, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 h, l;
        split_bf16((float)rb[p][e], h, l);
        hi[e] = h;
        lo[e] = l;
      }
      *reinterpret_cast<v8bf*>(&Bh[buf][q * LDK + 8 * kg]) = hi;
      *reinterpret_cast<v8bf*>(&Bl[buf][q * LDK + 8 * kg]) = lo;
    }
  };
  auto compute = [&](int cur) {
    v8bf ah[FM], al[FM], bh[FQ], bl[FQ];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      ah[i] = *reinterpret_cast<const v8bf*>(&Ah[cur][(wm0 + i * 16 + lr) * LDK + 8 * lk]);
      al[i] = *reinterpret_cast<const v8bf*>(&Al[cur][(wm0 + i * 16 + lr) * LDK + 8 * lk]);
    }
#pragma unroll
    for (int j = 0; j < FQ; ++j) {
      bh[j] = *reinterpret_cast<const v8bf*>(&Bh[cur][(wq0 + j * 16 + lr) * LDK + 8 * lk]);
      bl[j] = *reinterpret_cast<const v8bf*>(&Bl[cur][(wq0 + j * 16 + lr) * LDK + 8 * lk]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FQ; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[i][j], 0, 0, 0);
      }
  };
  const int nk = (Ki + KC - 1) / KC;
  TA ra0[AG][8], ra1[AG][8];
  TB rb0[BG][8], rb1[BG][8];
  gload(ra0, rb0, 0);
  gload(ra1, rb1, KC);
  sstore(ra0, rb0, 0);
  __syncthreads();
  int kc = 0;
  for (; kc + 2 < nk; kc += 2) {
    gload(ra0, rb0, (kc + 2) * KC);
    compute(0);
    sstore(ra1, rb1, 1);
    __syncthreads();
    gload(ra1, rb1, (kc + 3) * KC);
    compute(1);
    sstore(ra0, rb0, 0);
    __syncthreads();
  }
  compute(0);
  if (kc + 1 < nk) {
    sstore(ra1, rb1, 1);
    __syncthreads();
    compute(1);
  }
  const long cbase = b * g.sC;
  lp_store_tile<OUT32, false>(g.epi, [&](auto&& f) {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int m = m0 + wm0 + i * 16 + lr;
      if (m >= Mi) continue;
#pragma unroll
      for (int j = 0; j < FQ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = q0 + wq0 + j * 16 + 4 * lk + r;
          if (q >= Qi) continue;
          f(cbase + m + g.ldc * (long)q, acc[i][j][r], 0.0f);
        }
    }
  });
}

template <int PREC, typename TA, typename TB, bool OUT32, bool BK, int TM, int TQ, int WGM, int WGQ>
int launch_lp_tile(GemmArgs& g, hipStream_t s) {
  set_tile_counts(g, TM, TQ);
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  if (nt <= 0) return EXPINT_OK;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "mode product: too many tiles (%ld)", nt);
  if constexpr (PREC == EXPINT_PREC_FP32)
    hipLaunchKernelGGL((k_mode_product_f32<TA, TB, OUT32, BK, TM, TQ, 16, WGM, WGQ>), dim3((unsigned)nt),
                       dim3(64 * WGM * WGQ), 0, s, g);
  else if (BK && (g.bq * (long)sizeof(TB)) % 16 == 0)
    hipLaunchKernelGGL((k_mode_product_bf16x3<TA, TB, OUT32, BK, TM, TQ, WGM, WGQ, BK>), dim3((unsigned)nt),
                       dim3(64 * WGM * WGQ), 0, s, g);
  else
    hipLaunchKernelGGL((k_mode_product_bf16x3<TA, TB, OUT32, BK, TM, TQ, WGM, WGQ>), dim3((unsigned)nt),
                       dim3(64 * WGM * WGQ), 0, s, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "mode product launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

// Tile shapes of the reduced-precision products (TMxTQ outputs, w = waves; "t":
// the waves split the tile 2 x 4 instead of 4 x 2).  bf16x3 stages one 8-element
// K group per thread and chunk, so TM and TQ are at least half the thread count.
const char* const kF32TileNames[] = {"128x64w8", "64x64w4", "128x128w8", "128x128w16", "256x128w16"};
const char* const kBf16TileNames[] = {"64x64w4", "128x128w8", "128x128w8t", "256x128w8", "128x256w8t"};
constexpr int kNumF32Tiles = 5, kNumBf16Tiles = 5;

// The autotuner's choice (or EXPINT_LP_TILE) comes first; defaults: FP32
// 128x64 on 8 waves (as FP64), bf16x3 64x64 on 4 waves.
template <int PREC, typename TA, typename TB, bool OUT32, bool BK>
int launch_lp_typed(GemmArgs& g, hipStream_t s) {
  const int c = tune_choice(TuneKey{PREC == EXPINT_PREC_FP32 ? TUNE_LP_FP32 : TUNE_LP_BF16X3, g.M, g.Q, g.K, g.batches});
  if constexpr (PREC == EXPINT_PREC_FP32) {
    switch (c) {
      case 1: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 64, 64, 2, 2>(g, s);
      case 2: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 128, 4, 2>(g, s);
      case 3: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 128, 4, 4>(g, s);
      case 4: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 256, 128, 4, 4>(g, s);
      default: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 64, 4, 2>(g, s);
    }
  } else {
    switch (c) {
      case 1: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 128, 4, 2>(g, s);
      case 2: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 128, 2, 4>(g, s);
      case 3: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 256, 128, 4, 2>(g, s);
      case 4: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 128, 256, 2, 4>(g, s);
      default: return launch_lp_tile<PREC, TA, TB, OUT32, BK, 64, 64, 2, 2>(g, s);
    }
  }
}

// V (FP64 or FP32) and M (FP64) in; out0 FP32 (plain store) or the FP64 epilogue.
template <int PREC, bool OUT32>
int launch_lp_prec(bool v32, GemmArgs& g, bool mode1, hipStream_t s) {
  if (mode1)  // Aop = M (FP64), Bop = V
    return v32 ? launch_lp_typed<PREC, double, float, OUT32, true>(g, s)
               : launch_lp_typed<PREC, double, double, OUT32, true>(g, s);
  // Aop = V slab, Bop = M^T (FP64)
  return v32 ? launch_lp_typed<PREC, float, double, OUT32, false>(g, s)
             : launch_lp_typed<PREC, double, double, OUT32, false>(g, s);
}

// complex data, FP32 contraction (complex64 arithmetic): 4 FP32 MFMAs per block
template <typename TA, typename TB, bool OUT32, bool BK>
int launch_c64_typed(GemmArgs& g, hipStream_t s) {
  constexpr int TM = 64, TQ = 64;
  set_tile_counts(g, TM, TQ);
  const long nt = g.tiles_m * g.tiles_q * g.batches;
  if (nt <= 0) return EXPINT_OK;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "mode product: too many tiles (%ld)", nt);
  hipLaunchKernelGGL((k_mode_product_f32<TA, TB, OUT32, BK, TM, TQ, 16, 2, 4>), dim3((unsigned)nt), dim3(512), 0, s, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "mode product launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

template <bool OUT32>
int launch_c64(bool v32, GemmArgs& g, bool mode1, hipStream_t s) {
  if (mode1)
    return v32 ? launch_c64_typed<cdouble, cfloat, OUT32, true>(g, s)
               : launch_c64_typed<cdouble, cdouble, OUT32, true>(g, s);
  return v32 ? launch_c64_typed<cfloat, cdouble, OUT32, false>(g, s)
             : launch_c64_typed<cdouble, cdouble, OUT32, false>(g, s);
}

}  // namespace

int lp_tile_count(int precision) { return precision == EXPINT_PREC_FP32 ? kNumF32Tiles : kNumBf16Tiles; }
const char* lp_tile_name(int precision, int i) {
  if (i < 0 || i >= lp_tile_count(precision)) return "?";
  return precision == EXPINT_PREC_FP32 ? kF32TileNames[i] : kBf16TileNames[i];
}

TuneKey lp_key(int precision, long s, int n, long r) {
  const int fam = precision == EXPINT_PREC_FP32 ? TUNE_LP_FP32 : TUNE_LP_BF16X3;
  if (s == 1) return TuneKey{fam, n, r, n, 1};
  return TuneKey{fam, s, n, n, r};
}

int launch_mode_product_lp(int precision, bool cplx, bool v32, bool out32, long s, int n, long r, const void* M,
                           const void* V, const Epilogue& epi, void* stream) {
  if (s <= 0 || n <= 0 || r <= 0) return EXPINT_OK;
  const long bytes = s * (long)n * r * (cplx ? 16 : 8);
  if (bytes >= (1L << 31))
    return set_error(EXPINT_ENOTSUP, "mode product: tensors of %ld bytes exceed the 2 GiB limit", bytes);
  if (out32 && (epi.op != EPI_AXPBY || epi.alpha != 1.0 || epi.beta != 0.0))
    return set_error(EXPINT_EINVAL, "reduced-precision intermediate modes only store plainly");
  GemmArgs g;
  g.epi = epi;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool mode1 = s == 1;
  if (mode1) {
    g.A = M; g.lda = n; g.B = V; g.bk = 1; g.bq = n;
    g.M = n; g.Q = r; g.K = n; g.sA = 0; g.sC = 0; g.ldc = n; g.batches = 1;
  } else {
    g.A = V; g.lda = s; g.B = M; g.bk = n; g.bq = 1;
    g.M = s; g.Q = n; g.K = n; g.sA = s * (long)n; g.sC = s * (long)n; g.ldc = s; g.batches = r;
  }
  if (cplx) {
    if (precision != EXPINT_PREC_FP32)
      return set_error(EXPINT_ENOTSUP, "complex data: reduced precision is FP32 (complex64) only");
    return out32 ? launch_c64<true>(v32, g, mode1, st) : launch_c64<false>(v32, g, mode1, st);
  }
  if (precision == EXPINT_PREC_FP32)
    return out32 ? launch_lp_prec<EXPINT_PREC_FP32, true>(v32, g, mode1, st)
                 : launch_lp_prec<EXPINT_PREC_FP32, false>(v32, g, mode1, st);
  if (precision == EXPINT_PREC_BF16X3)
    return out32 ? launch_lp_prec<EXPINT_PREC_BF16X3, true>(v32, g, mode1, st)
                 : launch_lp_prec<EXPINT_PREC_BF16X3, false>(v32, g, mode1, st);
  return set_error(EXPINT_ENOTSUP, "unknown contraction precision %d", precision);
}

}  // namespace expint
