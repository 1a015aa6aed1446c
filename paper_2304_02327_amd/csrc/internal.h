// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/expint.h"

namespace expint {

// records a thread-local message and returns `code`
int set_error(int code, const char* fmt, ...);

// Argument checks shared by the entry points (host_abi.cpp): the total N of a
// shape (d <= 4, every n >= 1, N < 2^31), the operand limits of the kernels
// (each tensor below 2 GiB; exact slice: n_mu <= kSliceMaxK and digit planes
// below 2 GiB), whether a precision code is known, and the workspace layout of
// tucker_apply (ping-pong tensors, the tensor digits of the largest mode, the
// digits of every M).
int validate_shape(int d, const int* n, long* N);
int check_operand_limits(int d, const int* n, long N, int dtype, int precision);
bool valid_precision(int precision);
int tucker_ws_layout(int d, const int* n, long N, int dtype, int precision, int modes, size_t* tensors,
                     size_t* digits, size_t* mdigits);
size_t sliced_tensor_digits_bytes(int d, const int* n, long N);

int phi_setup_real(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo);
int phi_setup_complex(int n, const double* A, int lda, double tau, int ell_max, double* out, int ldo);
// phi_0..phi_ell_max of tau A by EXPINT_PHI_TAYLOR or EXPINT_PHI_QUAD (complex: interleaved)
int phi_setup_method(int method, bool cplx, int n, const double* A, int lda, double tau, int ell_max, double* out,
                     int ldo);
// keep this thread's phi_setup calls on one host thread (callers that already parallelise)
void phi_setup_single_threaded(bool on);

// ---------------------------------------------------------------------------
// launch-configuration tuning (the autotuner, tune.hip)
// ---------------------------------------------------------------------------

// A family is a kernel whose launch configuration (tile shape, waves, pipeline
// depth; for modes 1 and 2 also "not fused") has several candidates, all of
// which compute the same sums in the same order; a key is one launch shape.
enum TuneFamily : int {
  TUNE_MP_REAL = 0,  // FP64 mu-mode product, real data     key (M, Q, K, batches)
  TUNE_MP_CPLX = 1,  // FP64 mu-mode product, complex data  key (M, Q, K, batches)
  TUNE_SLICED = 2,   // exact-slice int8 product            key (M, Q, Kpad, batches)
  TUNE_MODES12 = 3,  // modes 1 and 2 in one launch         key (n1, n2, r, 0); last candidate = not fused
  TUNE_LP_FP32 = 4,  // FP32 mu-mode product (real data)    key (M, Q, K, batches)
  TUNE_LP_BF16X3 = 5,  // bf16x3 mu-mode product            key (M, Q, K, batches)
  TUNE_GROUPED = 6,  // grouped tile scheme of a batched phase  key (scheme/phase, count, total, size hash)
  TUNE_FAMILIES = 7
};
struct TuneKey {
  int family = 0;
  long a = 0, b = 0, c = 0, d = 0;
};
int tune_candidate_count(int family);
const char* tune_candidate_name(int family, int i);
// The candidate a launch of shape k uses: one forced by the tuner on this
// thread, else the environment override of the family (EXPINT_TILE,
// EXPINT_SLICE_TILE, EXPINT_M12), else the tuned choice, else -1 (the
// launcher's own measured default).
int tune_choice(const TuneKey& k);
// The tuned choice of k alone (-1 if none).
int tune_lookup(const TuneKey& k);
// Times every candidate of k's family (each call of `launch` makes the launches
// of the candidate tune_choice(k) returns while it runs) and keeps the fastest;
// a key tuned before is not timed again.
int tune_key(const TuneKey& k, void* stream, const std::function<int()>& launch);
// Keys of the launches the kernels make for a mu-mode product of a tensor viewed
// as (s, n, r), and for modes 1 and 2 of an n1 x n2 x r stack.
TuneKey mode_product_key(bool cplx, long s, int n, long r);
TuneKey sliced_key(long s, int n, long r);
TuneKey modes12_key(int n1, int n2, long r);
TuneKey lp_key(int precision, long s, int n, long r);
// Tunes every launch a Tucker operator of this shape, element type and
// contraction precision makes (all modes present), on scratch tensors;
// synchronous, allocates and frees its scratch.
int tune_tucker_shapes(int d, const int* n, int dtype, int precision, void* stream);
// "family a b c d: candidate (tuned, us)" or ": default" for one key
std::string tune_describe(const TuneKey& k);
// Candidate names of each family (defined next to the kernels).
int mode_product_tile_count();
const char* mode_product_tile_name(int i);
int sliced_tile_count();
const char* sliced_tile_name(int i);
int modes12_shape_count();
const char* modes12_shape_name(int i);
int lp_tile_count(int precision);
const char* lp_tile_name(int precision, int i);

// ---------------------------------------------------------------------------
// mu-mode product launcher
// ---------------------------------------------------------------------------

// Grid and clock of a coordinate- and time-dependent nonlinearity
// (EXPINT_G_ADR_PAPER): x_mu = (i_mu + 1) h_mu; t_n = clock[0] + clock[1] tau
// with clock a device pair {t0, steps taken} advanced by a kernel each step.
struct GridTime {
  int n[3] = {1, 1, 1};
  double h[3] = {0.0, 0.0, 0.0};
  double eps = 0.0, alpha = 0.0;
  const double* clock = nullptr;
  double tau = 0.0;
};

// What the last stage of a mu-mode product does with its result Y (per
// element e of the tensor; every tensor shares the layout of Y).
enum EpiOp : int {
  EPI_AXPBY = 0,        // out0[e] = alpha * Y + beta * out0[e]   (beta == 0: out0 not read)
  EPI_EXP_EULER = 1,    // out0[e] = in1[e] + Y                   (U_{n+1} = U_n + P)
  EPI_ETD2RK_1 = 2,     // u = in1[e]; u2 = u + Y; out0[e] = u2; out1[e] = tau (g(u2) - g(u))
  EPI_ETD2RK_2 = 3,     // out0[e] = in1[e] + c * Y
  EPI_LAWSON2B_2 = 4,   // out0[e] = Y + c * g(in1[e])           (c = tau / 2)
  EPI_LINEAR = 5,       // out0[e] = alpha Y + beta in1[e] + c in2[e]   (in1 / in2 optional)
  EPI_DIAG = 6,         // out0[e] = alpha Y + c [e mod ldiag == 0]: c added on the diagonal of a
                        // square matrix output with leading dimension ldiag - 1
};

struct Epilogue {
  int op = EPI_AXPBY;
  int g = EXPINT_G_NONE;
  double alpha = 1.0, beta = 0.0, tau = 0.0, c = 0.0, gparam = 0.0;
  void* out0 = nullptr;        // primary output (always written)
  const void* in1 = nullptr;   // secondary input
  const void* in2 = nullptr;   // third input (EPI_LINEAR)
  void* out1 = nullptr;        // secondary output
  long ldiag = 1;              // EPI_DIAG: n + 1 for an n x n column-major output
  GridTime gt;                 // for EXPINT_G_ADR_PAPER
};

// Y = V x_mu M for a tensor viewed as (s, n, r): s = prod_{nu<mu} n_nu (stride 1),
// n = n_mu, r = prod_{nu>mu} n_nu.  M is n x n column-major (device).  The
// epilogue decides what is stored.  dtype EXPINT_F64 or EXPINT_C128.
int launch_mode_product(int dtype, long s, int n, long r, const void* M, const void* V,
                        const Epilogue& epi, void* stream);

// Modes 1 and 2 of a Tucker operator in one launch (FP64, real data): for
// each of the r slabs V_b of n1 x n2 (first index fastest), M1 V_b M2^T goes
// through the epilogue at the slab's own positions.  M1 and M2 are n1 x n1 and
// n2 x n2 column-major (device).  The output must not overlap V.
constexpr int kModes12MaxN1 = 4096, kModes12MaxN2 = 128;
bool modes12_fits(int n1, int n2);
int launch_modes12(int n1, int n2, long r, const void* M1, const void* M2, const void* V, const Epilogue& epi,
                   void* stream);

// Grouped FP64 GEMMs in one launch (batched instances).  A descriptor
// describes C[m, q] = sum_k A[m + lda k] B[k bk + q bq] for m < M, q < Q,
// k < K with output element m + ldc q and an epilogue; bk == 1 (B contiguous
// along k) or bq == 1 (contiguous along q) selects the kernel.  A workgroup map
// (grouped_block_map) assigns the tiles to the workgroups.
size_t gemm_desc_size();
// gate (device int, optional): the descriptor's tiles run only while *gate > gate_level
int make_gemm_desc(void* out, const void* A, long lda, const void* B, long bk, long bq, long M, long Q, long K,
                   long ldc, const Epilogue& epi, const int* gate = nullptr, int gate_level = 0);
long gemm_desc_tiles(const void* desc);
// Grouped tile schemes (which GEMMs of a launch take the larger tile class):
// set a descriptor's class and tile counts for a scheme (make_gemm_desc sets scheme 0).
int grouped_scheme_count();
const char* grouped_scheme_name(int i);
void gemm_desc_set_scheme(void* desc, int scheme);
// Workgroup b of a grouped launch runs tile `tile` of descriptor `desc` (none if desc < 0).
struct GroupedBlock {
  int desc, tile;
};
// The map of `count` consecutive descriptors (host) under a grouped scheme: each
// GEMM's tiles on one XCD, balanced by the scheme's work measure.
void grouped_block_map(const void* descs, int count, int scheme, std::vector<GroupedBlock>& map);
bool grouped_block_map_valid(const void* descs, int count, const std::vector<GroupedBlock>& map);
// descs and map (blocks entries) in device memory; every descriptor follows `scheme`.
int launch_grouped_gemm(bool bk_contiguous, const void* descs, const GroupedBlock* map, long blocks, int scheme,
                        void* stream);

// Fused time stepping of a small two-dimensional FP64 problem (n1, n2 <= 64):
// one workgroup runs nsteps steps with the state in LDS.  M[mu][l] are the
// device phi_l(tau A_mu) the scheme uses; K u comes from the stencil
// coefficients (3 x n per direction, sub / diag / super) or the dense A_mu.
struct SmallArgs {
  double* U = nullptr;
  const double* M[2][3] = {};
  const double* stc[2] = {};
  int periodic[2] = {0, 0};
  const double* A[2] = {};
  int stencil = 0;
  int n1 = 1, n2 = 1;
  double tau = 0.0, gparam = 0.0;
  int scheme = 0, g = 0;
  int nsteps = 0;
};
bool small2d_fits(int d, const int* n);
int launch_small2d(const SmallArgs& a, void* stream);

// Exact-slice contraction (EXPINT_PREC_SLICED): each operand fibre is cut
// into kSliceDigits balanced base-254 digits under one power-of-two exponent
// and the digit products run exactly on int8 MFMA.  A digit buffer holds the
// planes of `rows` fibres padded to slice_kpad(n) followed by their exponents.
constexpr int kSliceDigits = 5;
constexpr int kSliceProducts = 19;  // digit pairs (i, j) with i + j <= kSliceDigits
constexpr int kSliceMaxK = 26624;  // longest contraction whose int32 level sums stay exact
int slice_kpad(int n);
size_t slice_digits_bytes(long rows, int n);
// digits of the fibres along the middle index of V viewed as (s, n, r);
// contiguous == true requires s == 1 (mode 1)
int launch_slice(const double* V, long s, int n, long r, bool contiguous, void* out, void* stream);
// mu-mode product from digit buffers: Mdig holds the n rows of M (launch_slice
// of M viewed as (n, n, 1)), Vdig the fibres of V; mode1 selects the roles of
// mode 1 (contiguous V fibres) or of the modes >= 2
int launch_sliced_mode_product(long s, int n, long r, bool mode1, const void* Mdig, const void* Vdig,
                               const Epilogue& epi, void* stream);

// Reduced-precision contraction (EXPINT_PREC_FP32 / EXPINT_PREC_BF16X3; complex
// data FP32 only) of a mu-mode product: V is FP32 (complex64) when v32, else
// FP64 (complex128), M is FP64 / complex128; with out32 the result is stored
// plainly in single precision into epi.out0, else it runs the FP64 epilogue.
int launch_mode_product_lp(int precision, bool cplx, bool v32, bool out32, long s, int n, long r, const void* M,
                           const void* V, const Epilogue& epi, void* stream);

// ---------------------------------------------------------------------------
// pointwise / stencil launchers
// ---------------------------------------------------------------------------

// Per-direction 3-point stencil coefficients on the device: lo[i] = A[i, i-1],
// di[i] = A[i, i], up[i] = A[i, i+1]; with `periodic` the neighbours wrap
// (lo[0] = A[0, n-1], up[n-1] = A[n-1, 0]).  Complex data: interleaved.
struct Stencil {
  int d = 0;
  int n[4] = {1, 1, 1, 1};
  const void* coef[4] = {nullptr, nullptr, nullptr, nullptr};  // 3 * n[mu] elements: lo | di | up
  int periodic[4] = {0, 0, 0, 0};
  // Every direction Toeplitz (constant diagonals): the three values of each
  // direction travel as kernel arguments, interleaved (re, im) for complex data.
  bool toeplitz = false;
  double tc[4][3][2] = {};
};

// W = tau * (K U + g(t_n, U)) with K applied as the stencil.
int launch_stage_stencil(int dtype, const Stencil& st, long N, const void* U, void* W,
                         double tau, int g, double gparam, const GridTime& gt, void* stream);
// W = a * g(t_n, U) (no K term; the dense path adds tau * U x_mu A_mu afterwards)
int launch_scaled_g(int dtype, long N, const void* U, void* W, double a, int g, double gparam,
                    const GridTime& gt, void* stream);
// Wa = U + tau g(t_n, U); Wb = U + tau/2 g(t_n, U) (Wb may be NULL)
int launch_lawson_stage(int dtype, long N, const void* U, void* Wa, void* Wb, double tau, int g,
                        double gparam, const GridTime& gt, void* stream);
// clock = {t0, 0} / clock[1] += 1 (one thread; graph-capturable, no memset)
int launch_clock_set(double* clock, double t0, void* stream);
int launch_clock_tick(double* clock, void* stream);
// flag[0] |= 1 if any of count doubles at x is not finite (flag: device int)
int launch_finite_check(const double* x, long count, int* flag, void* stream);

}  // namespace expint
