// Modes 1 and 2 of a Tucker operator in one launch (FP64, real data).
//
// Seen as a stack of r = n_3 ... n_d slabs V_b = V(:, :, b) of n1 x n2, the
// first two mu-mode products of the chain (eq. tuckerexp) map every slab to
// P_b = M1 V_b M2^T.  A workgroup owns RM rows of one slab's result: it
// forms T = M1(rows, :) V_b on FP64 MFMA, keeps T in LDS and multiplies it by
// M2^T there, so the intermediate tensor between the two modes never goes to
// HBM and one launch does the work of two.  The flops are those of the two
// separate products.  The row blocks of a slab are neighbouring tiles, which
// xcd_remap keeps on one XCD, so the slab's readers share that XCD's L2.
//
// Each K loop (n1 for the first product, n2 for the second) runs in chunks of
// KC through two LDS buffers with two register sets in flight, one barrier
// per chunk, as the single-mode kernel does.  Operands are read with buffer
// loads whose resource covers exactly one operand (M1, M2 or the slab), so a
// row, column or K index past the end reads zero.

#include <cstdlib>
#include <cstring>

#include "internal.h"
#include "tile_common.h"

namespace expint {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

struct Modes12Args {
  const double* M1;  // n1 x n1, column-major
  const double* M2;  // n2 x n2, column-major
  const double* V;   // n1 x n2 x r, first index fastest
  int n1, n2;
  long r, row_tiles;
  Epilogue epi;
};

__device__ __forceinline__ double bld(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// NQ: columns of the slab a workgroup covers (n2 <= NQ); RM rows per
// workgroup; WGM x 4 waves, each owning RM / WGM rows and NQ / 4 columns of T
// and of the result.
// SCHED 0: the compiler's instruction order.  1: a wave raises its issue
// priority while it has MFMAs to issue (s_setprio), so the waves of a SIMD that
// are staging chunks yield the issue slots to one that multiplies.  2: each
// chunk's MFMAs are interleaved with its LDS reads, LDS writes and global
// loads (scheduling groups).
template <int NQ, int RM, int WGM, int SCHED = 0>
__global__ __launch_bounds__(256 * WGM) void k_modes12(Modes12Args g) {
  constexpr int KC = 16, NW = 4 * WGM, NT = 64 * NW;
  constexpr int WM = RM / WGM, WQ = NQ / 4, FQ = WQ / 16, FM = WM / 16;
  constexpr int LDA = RM;      // M1 chunk: As[k * LDA + m]
  constexpr int LDB = NQ + 1;  // V_b or M2^T chunk: Bs[k * LDB + q], odd for the transposed stores
  constexpr int LDT = RM;      // T: Ts[j * LDT + m]
  constexpr int AL = RM * KC / NT, BL = NQ * KC / NT;
  constexpr unsigned SZ = 8;
  static_assert(FM >= 1 && WM % 16 == 0 && FQ >= 1 && WQ % 16 == 0 && AL * NT == RM * KC && BL * NT == NQ * KC,
                "bad shape");
  __shared__ double As[2][KC * LDA];
  __shared__ double Bs[2][KC * LDB];
  __shared__ double Ts[NQ * LDT];

  const long nt = g.row_tiles * g.r;
  const long t = xcd_remap((long)blockIdx.x, nt);
  const long b = t / g.row_tiles;
  const int i0 = (int)(t % g.row_tiles) * RM;
  const int n1 = g.n1, n2 = g.n2;
  const unsigned m1bytes = (unsigned)n1 * (unsigned)n1 * SZ;
  const unsigned m2bytes = (unsigned)n2 * (unsigned)n2 * SZ;
  const unsigned vbytes = (unsigned)n1 * (unsigned)n2 * SZ;
  const __amdgpu_buffer_rsrc_t rm1 = make_rsrc(g.M1, m1bytes);
  const __amdgpu_buffer_rsrc_t rm2 = make_rsrc(g.M2, m2bytes);
  const __amdgpu_buffer_rsrc_t rv = make_rsrc(g.V + b * (long)n1 * n2, vbytes);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm0 = (wave % WGM) * WM, wq0 = (wave / WGM) * WQ;

  // Per-thread byte offsets of the chunk at k0 = 0 (the chunk advance is the
  // scalar offset).  Rows of M1 past n1 and columns past n2 point at the end
  // of their resource; a K index past the end lands there by itself for M1
  // and M2 and is redirected per chunk for the slab.
  unsigned oa[AL], ov[BL], om[BL];
#pragma unroll
  for (int p = 0; p < AL; ++p) {
    const int idx = tid + NT * p, m = idx % RM, k = idx / RM;
    oa[p] = (i0 + m < n1) ? ((unsigned)(i0 + m) + (unsigned)n1 * (unsigned)k) * SZ : m1bytes;
  }
#pragma unroll
  for (int p = 0; p < BL; ++p) {
    const int idx = tid + NT * p;
    const int k = idx % KC, j = idx / KC;  // slab chunk, k fastest
    ov[p] = (j < n2) ? ((unsigned)k + (unsigned)n1 * (unsigned)j) * SZ : vbytes;
    const int q = idx % NQ, kq = idx / NQ;  // M2^T chunk, q fastest: M2[q + n2 k]
    om[p] = (q < n2) ? ((unsigned)q + (unsigned)n2 * (unsigned)kq) * SZ : m2bytes;
  }

  v4d acc[FM][FQ];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FQ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  // ---- T = M1(rows, :) V_b ------------------------------------------------
  auto load1 = [&](double (&a)[AL], double (&v)[BL], int c) {
    const unsigned k0 = (unsigned)(c * KC);
#pragma unroll
    for (int p = 0; p < AL; ++p) a[p] = bld(rm1, oa[p], (unsigned)n1 * k0 * SZ);
#pragma unroll
    for (int p = 0; p < BL; ++p) {
      const unsigned k = (unsigned)((tid + NT * p) % KC);
      v[p] = bld(rv, (k0 + k < (unsigned)n1) ? ov[p] : vbytes, k0 * SZ);
    }
  };
  auto store1 = [&](const double (&a)[AL], const double (&v)[BL], int buf) {
#pragma unroll
    for (int p = 0; p < AL; ++p) {
      const int idx = tid + NT * p;
      As[buf][(idx / RM) * LDA + idx % RM] = a[p];
    }
#pragma unroll
    for (int p = 0; p < BL; ++p) {
      const int idx = tid + NT * p;
      Bs[buf][(idx % KC) * LDB + idx / KC] = v[p];
    }
  };
  auto compute1 = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double af[FM], bf[FQ];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = As[buf][(kk + lk) * LDA + wm0 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < FQ; ++j) bf[j] = Bs[buf][(kk + lk) * LDB + wq0 + j * 16 + lr];
      if constexpr (SCHED == 1) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FQ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
      if constexpr (SCHED == 1) __builtin_amdgcn_s_setprio(0);
    }
  };

  // SCHED == 2: one chunk's work in a scheduling region, each MFMA followed by
  // its share of LDS reads, then an LDS write and a global load while they last
  auto interleave = [](int nvmem, int nwrite) {
    if constexpr (SCHED == 2) {
      constexpr int NM = FM * FQ * (KC / 4), NR = (FM + FQ) * (KC / 4);
      constexpr int RPM = (NR + NM - 1) / NM;
#pragma unroll
      for (int u = 0; u < NM; ++u) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);    // MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, RPM, 0);  // LDS read
        if (u < nwrite) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS write
        if (u < nvmem) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global load
      }
    }
  };
  const int nk1 = (n1 + KC - 1) / KC, nk2 = (n2 + KC - 1) / KC;
  double ra[2][AL], rb[2][BL];
  load1(ra[0], rb[0], 0);
  load1(ra[1], rb[1], 1);
  store1(ra[0], rb[0], 0);
  __syncthreads();
  int kc = 0;
  for (; kc + 2 < nk1; kc += 2) {
    load1(ra[0], rb[0], kc + 2);
    compute1(0);
    store1(ra[1], rb[1], 1);
    interleave(AL + BL, AL + BL);
    __syncthreads();
    load1(ra[1], rb[1], kc + 3);
    compute1(1);
    store1(ra[0], rb[0], 0);
    interleave(AL + BL, AL + BL);
    __syncthreads();
  }
  compute1(0);
  if (kc + 1 < nk1) {
    store1(ra[1], rb[1], 1);
    __syncthreads();
    compute1(1);
  }

  // ---- P = T M2^T -----------------------------------------------------------
  auto load2 = [&](double (&v)[BL], int c) {
    const unsigned k0 = (unsigned)(c * KC);
#pragma unroll
    for (int p = 0; p < BL; ++p) v[p] = bld(rm2, om[p], (unsigned)n2 * k0 * SZ);
  };
  auto store2 = [&](const double (&v)[BL], int buf) {
#pragma unroll
    for (int p = 0; p < BL; ++p) {
      const int idx = tid + NT * p;
      Bs[buf][(idx / NQ) * LDB + idx % NQ] = v[p];
    }
  };
  auto compute2 = [&](int buf, int c) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double af[FM], bf[FQ];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = Ts[(c * KC + kk + lk) * LDT + wm0 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < FQ; ++j) bf[j] = Bs[buf][(kk + lk) * LDB + wq0 + j * 16 + lr];
      if constexpr (SCHED == 1) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FQ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j], af[i], acc[i][j], 0, 0, 0);
      if constexpr (SCHED == 1) __builtin_amdgcn_s_setprio(0);
    }
  };

  // the first two M2^T chunks travel while T goes to LDS; acc[i][j][r] holds
  // T[wm0 + 16 i + lane mod 16, wq0 + 16 j + lane / 16 + 4 r]
  load2(rb[0], 0);
  load2(rb[1], 1);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FQ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Ts[(wq0 + j * 16 + lk + 4 * r) * LDT + wm0 + i * 16 + lr] = acc[i][j][r];
        acc[i][j][r] = 0.0;
      }
  __syncthreads();  // T is complete and every wave is done with the first product's buffers
  store2(rb[0], 0);
  __syncthreads();
  kc = 0;
  for (; kc + 2 < nk2; kc += 2) {
    load2(rb[0], kc + 2);
    compute2(0, kc);
    store2(rb[1], 1);
    interleave(BL, BL);
    __syncthreads();
    load2(rb[1], kc + 3);
    compute2(1, kc + 1);
    store2(rb[0], 0);
    interleave(BL, BL);
    __syncthreads();
  }
  compute2(0, kc);
  if (kc + 1 < nk2) {
    store2(rb[1], 1);
    __syncthreads();
    compute2(1, kc + 1);
  }

  // acc[i][j][r] holds P_b[i0 + wm0 + 16 i + lane mod 16, wq0 + 16 j + lane / 16 + 4 r]
  const long cbase = b * (long)n1 * n2;
  epilogue_tile<double>(g.epi, [&](auto&& f) {
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int m = i0 + wm0 + i * 16 + lr;
      if (m >= n1) continue;
#pragma unroll
      for (int j = 0; j < FQ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = wq0 + j * 16 + lk + 4 * r;
          if (q < n2) f(cbase + m + (long)n1 * q, acc[i][j][r]);
        }
    }
  });
}

}  // namespace

bool modes12_fits(int n1, int n2) { return n1 >= 1 && n1 <= kModes12MaxN1 && n2 >= 1 && n2 <= kModes12MaxN2; }

TuneKey modes12_key(int n1, int n2, long r) { return TuneKey{TUNE_MODES12, n1, n2, r, 0}; }

namespace {

// Workgroup shapes (rows x waves; "p": s_setprio around the MFMAs, "i": the
// interleaved chunk schedule); EXPINT_M12 set to a name overrides the default.
const char* const kShapeNames[] = {"r32w4",   "r32w8",   "r16w4",    "r64w8",    "r64w16",
                                   "r32w8p", "r32w8i", "r64w16p", "r64w16i"};
constexpr int kRows[] = {32, 32, 16, 64, 64, 32, 32, 64, 64};
constexpr int kNumShapes = sizeof(kRows) / sizeof(kRows[0]);

// Measured on MI355X (FP64): at 128^3 the fused launch takes 24.8 us with 64
// rows on 16 waves and the interleaved chunk schedule ("r64w16i"), 26.0 us
// without it, 27.2 / 28.5 us with 32 rows on 8 waves (with / without), 29.0 us
// with 32 rows on 4 waves; at 80 x 81 x 82, where 64-row tiles give fewer
// workgroups than CUs, 32 rows on 8 waves is fastest.
// The autotuner's choice (or EXPINT_M12) comes first; its "not fused" candidate
// is decided before this launcher is called.
int shape_choice(int n1, int n2, long r) {
  const int c = tune_choice(modes12_key(n1, n2, r));
  if (c >= 0 && c < kNumShapes) return c;
  return (n1 + 63) / 64 * r >= 256 ? 8 : 6;
}

template <int NQ>
void launch_shape(int shape, long nt, hipStream_t st, const Modes12Args& g) {
  switch (shape) {
    case 1: hipLaunchKernelGGL((k_modes12<NQ, 32, 2>), dim3((unsigned)nt), dim3(512), 0, st, g); break;
    case 2: hipLaunchKernelGGL((k_modes12<NQ, 16, 1>), dim3((unsigned)nt), dim3(256), 0, st, g); break;
    case 3: hipLaunchKernelGGL((k_modes12<NQ, 64, 2>), dim3((unsigned)nt), dim3(512), 0, st, g); break;
    case 4: hipLaunchKernelGGL((k_modes12<NQ, 64, 4>), dim3((unsigned)nt), dim3(1024), 0, st, g); break;
    case 5: hipLaunchKernelGGL((k_modes12<NQ, 32, 2, 1>), dim3((unsigned)nt), dim3(512), 0, st, g); break;
    case 6: hipLaunchKernelGGL((k_modes12<NQ, 32, 2, 2>), dim3((unsigned)nt), dim3(512), 0, st, g); break;
    case 7: hipLaunchKernelGGL((k_modes12<NQ, 64, 4, 1>), dim3((unsigned)nt), dim3(1024), 0, st, g); break;
    case 8: hipLaunchKernelGGL((k_modes12<NQ, 64, 4, 2>), dim3((unsigned)nt), dim3(1024), 0, st, g); break;
    default: hipLaunchKernelGGL((k_modes12<NQ, 32, 1>), dim3((unsigned)nt), dim3(256), 0, st, g); break;
  }
}

}  // namespace

int modes12_shape_count() { return kNumShapes; }
const char* modes12_shape_name(int i) { return i >= 0 && i < kNumShapes ? kShapeNames[i] : "?"; }

int launch_modes12(int n1, int n2, long r, const void* M1, const void* M2, const void* V, const Epilogue& epi,
                   void* stream) {
  if (r <= 0) return EXPINT_OK;
  if (!modes12_fits(n1, n2))
    return set_error(EXPINT_EINVAL, "fused modes 1 and 2: n1 = %d, n2 = %d outside 1..%d, 1..%d", n1, n2,
                     kModes12MaxN1, kModes12MaxN2);
  const int shape = shape_choice(n1, n2, r);
  Modes12Args g;
  g.M1 = static_cast<const double*>(M1);
  g.M2 = static_cast<const double*>(M2);
  g.V = static_cast<const double*>(V);
  g.n1 = n1;
  g.n2 = n2;
  g.r = r;
  g.row_tiles = (n1 + kRows[shape] - 1) / kRows[shape];
  g.epi = epi;
  const long nt = g.row_tiles * r;
  if (nt > 0x7fffffffL) return set_error(EXPINT_EINVAL, "fused modes 1 and 2: too many tiles (%ld)", nt);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (n2 <= 64)
    launch_shape<64>(shape, nt, st, g);
  else
    launch_shape<128>(shape, nt, st, g);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return set_error(EXPINT_EHIP, "fused modes 1 and 2 launch failed: %s", hipGetErrorString(err));
  return EXPINT_OK;
}

}  // namespace expint
