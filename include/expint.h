/*
 * expint.h -- C ABI of the direction-split ("phisplit") exponential-integrator
 * library for AMD Instinct MI355X (gfx950).
 *
 * Problem (paper section 1, eqs. ODE and kronsum):
 *     u'(t) = K u(t) + g(t, u(t)),   K = A_d (+) ... (+) A_1 = sum_mu I (x) .. (x) A_mu (x) .. (x) I,
 * with u = vec(U) for an order-d tensor U of size n_1 x ... x n_d.
 *
 * Conventions shared by every entry point:
 *   - Layout: tensors are stored with the first index fastest (vec() stacks
 *     columns, section 1 after eq. tuckerexp); element (i_1,..,i_d) sits at
 *     i_1 + n_1 (i_2 + n_2 (i_3 + ...)).  Small matrices are column-major.
 *     Complex data is interleaved (re, im) doubles.
 *   - Memory: pointers documented as "device" must be device memory of the
 *     current HIP device, 16-byte aligned; "host" pointers are ordinary host
 *     memory.  The caller owns every buffer it passes and keeps it alive until
 *     the work on the given stream has completed.  The library never frees
 *     caller memory.  A plan owns only its own small device copies of the
 *     phi matrices and stencil coefficients.
 *   - Streams: `stream` is a hipStream_t passed as void*; NULL is the legacy
 *     default stream.  Every entry point that takes a stream only enqueues
 *     work on it and returns without synchronising.
 *   - Errors: every int-returning function returns EXPINT_OK (0) or a negative
 *     status; no exception crosses the ABI.  All arguments are validated before
 *     any work is enqueued; on error nothing has been launched.
 *     expint_last_error() returns a thread-local message for the last failure.
 */
#ifndef EXPINT_H
#define EXPINT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define EXPINT_OK          0
#define EXPINT_EINVAL     -1  /* invalid argument (shape, pointer, size, enum) */
#define EXPINT_ENOMEM     -2  /* host or device allocation failed (plan creation only) */
#define EXPINT_EHIP       -3  /* a HIP runtime call failed */
#define EXPINT_ENOTSUP    -4  /* valid but unsupported combination */
#define EXPINT_ENUMERIC   -5  /* non-finite input to phi_setup; a Rosenbrock-Euler phi_1 that needed more
                                 squarings than its plan provides (expint_batch_status) */
#define EXPINT_ENONFINITE -6  /* a state holds inf or nan (expint_plan_check_finite, expint_batch_status) */

/* element types of U / V / W */
#define EXPINT_F64   0    /* double */
#define EXPINT_C128  1    /* double complex, interleaved */

/* contraction precision of the mu-mode products (phi matrices are always built in FP64) */
#define EXPINT_PREC_FP64    0
#define EXPINT_PREC_FP32    1   /* operands rounded to FP32, FP32 MFMA */
#define EXPINT_PREC_BF16X3  2   /* x = hi + lo (bf16, RNE); hi*hi + hi*lo + lo*hi, FP32 accumulate */
#define EXPINT_PREC_SLICED  3   /* exact-slice: every operand fibre (a row of M, a fibre of the
                                   tensor along the contracted mode) as 5 balanced base-254 int8
                                   digits under one power-of-two exponent; the 19 digit products
                                   a_i b_j with i + j <= 5 summed exactly in int32 on int8 MFMA
                                   and combined in FP64.  Error of one contraction at most
                                   2^-38.9 (max|v| sum|m| + max|m| sum|v|) + n 2^-44.3 max|m| max|v|
                                   over the contracted fibres; FP64 between modes */

/* time-stepping schemes (paper section 2; tensor forms in section 3.2) */
#define EXPINT_LAWSON_EULER  0  /* eq. lawsoneulertensor */
#define EXPINT_LAWSON2B      1  /* eq. lawson2tensor */
#define EXPINT_EXP_EULER     2  /* eq. expEulertensor, split phi_1 */
#define EXPINT_ETD2RK        3  /* eq. ETD2RKtensor with the (l!)^{d-1} split factor of eq. dsphi */
#define EXPINT_ROSENBROCK_EULER 4  /* eq. expRosEulertensor; batched Riccati plans only (phi_1 of the
                                      Jacobian directions rebuilt on the device at every step) */

/* nonlinearities g(u) (autonomous) */
#define EXPINT_G_NONE        0  /* g = 0 */
#define EXPINT_G_ALLEN_CAHN  1  /* g = u - u^3 */
#define EXPINT_G_U2_1MU      2  /* g = u^2 (1 - u) */
#define EXPINT_G_CUBIC_NLS   3  /* g = -i kappa |u|^2 u (complex only; kappa = g_param) */
#define EXPINT_G_ADR_PAPER   4  /* g(t, x, u) = 1/(1 + u^2) + Psi(t, x): the manufactured source of the
                                   advection-diffusion-reaction test of section 4.2 (eq. ADR) on the inner
                                   grid x_mu = (i + 1)/(n_mu + 1), d = 3, eps = g_param, alpha = g_param2;
                                   non-autonomous: uses t */

/* ------------------------------------------------------------------------ */
/* phi_setup: the small matrices phi_l(tau A) of one direction               */
/* ------------------------------------------------------------------------ */

/*
 * phi_setup -- phi_0(tau A), ..., phi_{ell_max}(tau A) for one n x n matrix
 * (definitions: section 1, eqs. integraldef / seriesdef; construction:
 * section 3.1, scaling by 2^s and the squaring recurrence eq. squarephi, with
 * a Taylor expansion of the scaled matrix in place of the quadrature).
 *   n       >= 1
 *   A       host, column-major, leading dimension lda >= n, float64
 *   tau     any finite real (tau = 0 gives phi_l = I / l!)
 *   ell_max 0..3
 *   phi_out host, (ell_max+1) column-major n x n blocks, block l starting at
 *           phi_out + l * ldphi * n, leading dimension ldphi >= n
 * Returns the raw phi_l(tau A); the split factor (l!)^{d-1} is applied by the
 * stepping code, not here.  Runs on the host CPU in FP64.
 * Errors: EINVAL (bad sizes / NULL), ENUMERIC (non-finite entries or tau).
 */
int phi_setup(int n, const double* A, int lda, double tau, int ell_max,
              double* phi_out, int ldphi);

/* phi_setup_z -- complex twin of phi_setup: A and phi_out hold interleaved
 * complex doubles (leading dimensions counted in complex elements). */
int phi_setup_z(int n, const double* A, int lda, double tau, int ell_max,
                double* phi_out, int ldphi);

/* Constructions of the phi matrices (section 3.1). */
#define EXPINT_PHI_TAYLOR 0  /* scale by 2^s (||.||_1 <= 1/2), Taylor series eq. seriesdef, eq. squarephi */
#define EXPINT_PHI_QUAD   1  /* the paper's: scale by 2^s (||.||_1 < 1); phi_0 = e^Y and, for l > 0,
                                eq. phiquad on 8 Gauss-Legendre-Lobatto nodes of [0, 1] with the
                                exponentials e^{(1-theta) Y} from diagonal Pade approximants; then
                                eq. squarephi */

/* phi_setup_ex -- phi_setup (dtype EXPINT_F64) or phi_setup_z (EXPINT_C128)
 * with the construction chosen by method (EXPINT_PHI_*); same arguments,
 * layout and errors, plus EINVAL for an unknown method or dtype.  Both
 * constructions agree to FP64 rounding. */
int phi_setup_ex(int n, const double* A, int lda, double tau, int ell_max, int method, int dtype,
                 double* phi_out, int ldphi);

/* ------------------------------------------------------------------------ */
/* tucker_apply: W = alpha * (V x_1 M_1 x_2 ... x_d M_d) + beta * W          */
/* ------------------------------------------------------------------------ */

/*
 * Tucker operator (section 1, eq. tuckerexp; the mu-mode product is the
 * contraction spelled out by eq. forloop: (V x_mu M)[..i_mu..] =
 * sum_j M[i_mu, j] V[..j..]).
 *   d          1..4
 *   n          host array of d sizes, n[mu] >= 1, prod n[mu] < 2^31
 *   M          host array of d device pointers; M[mu] is an n[mu] x n[mu]
 *              column-major matrix of the element type, or NULL for the
 *              identity (the mode is skipped)
 *   V          device input tensor (not modified); must not alias W
 *   W          device output tensor
 *   alpha,beta real scalars; beta == 0 means W is not read
 *   dtype      EXPINT_F64 or EXPINT_C128
 *   precision  EXPINT_PREC_FP64; EXPINT_PREC_FP32 (real or complex data):
 *              operands rounded to FP32, FP32 accumulation; (real data only)
 *              EXPINT_PREC_BF16X3: operands split into two bf16 parts, FP32
 *              accumulation -- both keep FP32 intermediates between modes and
 *              return FP64; EXPINT_PREC_SLICED (real data only, n[mu] <=
 *              26624): exact-slice digits on int8 MFMA, FP64 intermediates
 *   ws         device workspace of at least tucker_workspace_size() bytes
 *              (may be NULL when that size is 0)
 *   stream     hipStream_t
 * Modes are applied in the order 1..d.  Results are deterministic (no
 * atomics, fixed reduction order).
 */
int tucker_apply(int d, const int* n, const void* const* M, const void* V, void* W,
                 double alpha, double beta, int dtype, int precision,
                 void* ws, size_t ws_bytes, void* stream);

/*
 * tucker_apply_noalloc -- tucker_apply for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments and kernels as tucker_apply, without
 * ws / ws_bytes.  The intermediates tucker_workspace_size() would count live in
 * a fixed device array of EXPINT_NOALLOC_SCRATCH_BYTES bytes that the library
 * keeps on each device it runs on until the process ends.  Nothing is
 * allocated; the first call on a device looks up that device's array address.
 * Every call on one device shares the array, so calls that overlap on one
 * device (concurrent streams, or threads without ordering) race; calls
 * ordered on one stream are safe.  The array needs no clearing: each call
 * writes every scratch byte it reads.  Results equal tucker_apply's bitwise.
 * Errors: as tucker_apply, and ENOTSUP when the shape needs more scratch than
 * EXPINT_NOALLOC_SCRATCH_BYTES (e.g. FP64 tensors above 4 Mi elements with
 * three or more modes), before anything is enqueued.
 */
#define EXPINT_NOALLOC_SCRATCH_BYTES (64u << 20)
int tucker_apply_noalloc(int d, const int* n, const void* const* M, const void* V, void* W,
                         double alpha, double beta, int dtype, int precision, void* stream);

/*
 * tucker_tune -- the autotuner: times every candidate launch configuration
 * (tile shape, waves, pipeline depth, modes 1 and 2 in one launch or two) of
 * the FP64, FP32, bf16x3 and exact-slice mu-mode products, for
 * every launch a tucker_apply of this shape, element type and precision (all
 * modes present) makes, on scratch operands of the same sizes (hashed values), and
 * keeps the fastest per launch shape and device architecture for the rest of
 * the process.  Later tucker_apply / expint_step launches of those shapes use
 * it; a shape tuned before is not timed again.  With the environment variable
 * EXPINT_TUNE_CACHE naming a file, choices are read from it first and new ones
 * appended, so a later process makes the same choices.  The candidates of a
 * launch compute the same sums in the same order, so results do not depend on
 * the choice.  Environment overrides (EXPINT_TILE, EXPINT_SLICE_TILE,
 * EXPINT_M12, EXPINT_LP_TILE) still take precedence.  Synchronous; allocates and frees its
 * scratch (about three tensors).  Complex data contracted in FP32 (complex64)
 * has one configuration (nothing to tune).  Errors: EINVAL, ENOTSUP (as
 * tucker_apply), ENOMEM, EHIP.
 */
int tucker_tune(int d, const int* n, int dtype, int precision, void* stream);

/* tucker_workspace_size -- bytes of workspace tucker_apply needs for this
 * shape, element type and precision (every M non-NULL; fewer modes need no
 * more).  Errors: EINVAL for a bad shape, dtype or precision. */
int tucker_workspace_size(int d, const int* n, int dtype, int precision, size_t* bytes);

/* tucker_fuses_modes12 -- *fused = 1 if a Tucker operator of this shape, with
 * M_1 and M_2 both present, runs modes 1 and 2 as one launch: FP64 real data
 * at EXPINT_PREC_FP64 with n[1] <= 128 and n[0] <= 4096, d >= 2.  The launch
 * computes M_1 V_b M_2^T for every n[0] x n[1] slab V_b with the intermediate
 * in on-chip memory (the same sums in the same order as two mode products).
 * The environment variable EXPINT_FUSE12=0 turns it off; EXPINT_TILE, which
 * forces a single-mode tile shape, does too.  Errors: EINVAL for a bad shape,
 * dtype, precision or a NULL fused. */
int tucker_fuses_modes12(int d, const int* n, int dtype, int precision, int* fused);

/* ------------------------------------------------------------------------ */
/* plans and time stepping                                                   */
/* ------------------------------------------------------------------------ */

typedef struct expint_plan expint_plan;

typedef struct expint_problem {
  int d;                 /* 1..4 */
  int n[4];              /* n[0..d-1] */
  const double* A[4];    /* host, column-major n[mu] x n[mu] (complex: interleaved), lda = n[mu] */
  double tau;            /* constant step size */
  int scheme;            /* EXPINT_LAWSON_EULER .. EXPINT_ETD2RK */
  int nonlin;            /* EXPINT_G_* */
  double g_param;        /* kappa of EXPINT_G_CUBIC_NLS, eps of EXPINT_G_ADR_PAPER */
  double g_param2;       /* alpha of EXPINT_G_ADR_PAPER */
  int dtype;             /* EXPINT_F64 or EXPINT_C128 */
  int precision;         /* contraction precision of the Tucker operators (EXPINT_PREC_*;
                            complex data: FP64 or FP32 only); K u, g and the stage
                            combination stay FP64.  EXPINT_PREC_SLICED keeps int8
                            digits of every phi in the plan */
  int phi_method;        /* construction of the phi matrices: EXPINT_PHI_TAYLOR (0) or
                            EXPINT_PHI_QUAD */
  int tune;              /* 1: autotune the launch configuration of every mu-mode
                            product (and of modes 1 and 2 together) the plan's
                            steps make, at plan creation, as tucker_tune does;
                            0: the library's measured defaults, or earlier tuning
                            results for the same shapes */
} expint_problem;

/*
 * expint_plan_create -- build the phi matrices phi_l(tau A_mu) once for every
 * direction (section 3.1 / 4.2: computed once before the time stepping),
 * upload them and the operator data to the current device.  Directions with
 * bitwise-identical A share their phi.  A tridiagonal A_mu (optionally with
 * periodic corner entries) is applied to U as a 3-point stencil; any other
 * A_mu as a dense mu-mode product.
 * Errors: EINVAL, ENOTSUP, ENOMEM, EHIP.  On error *plan is set to NULL.
 */
int expint_plan_create(expint_plan** plan, const expint_problem* prob);

/* expint_plan_workspace_size -- device workspace bytes expint_step/run need. */
int expint_plan_workspace_size(const expint_plan* plan, size_t* bytes);

/*
 * expint_plan_set_phi -- replace phi_l(tau A_mu) of direction mu (0-based)
 * with a host matrix (column-major n[mu] x n[mu], the plan's element type),
 * e.g. to separate contraction error from phi error in tests.  Synchronous.
 */
int expint_plan_set_phi(expint_plan* plan, int mu, int ell, const double* host_phi);

/*
 * expint_step -- advance U (device, in place) by one step of the plan's
 * scheme from time t.  Enqueues a fixed kernel sequence on `stream`:
 * stage input (K U by stencil or mu-mode products, plus g), one Tucker
 * operator per stage with the stage combination and the next g fused into
 * the last mu-mode product.  No allocation, so it may be graph-captured.
 */
int expint_step(expint_plan* plan, void* U, double t, void* ws, void* stream);

/*
 * expint_run -- nsteps >= 0 steps from t0.  use_graph != 0 captures one step
 * into a HIP graph (once per plan / U / ws / stream combination) and replays
 * it nsteps times; use_graph == 0 enqueues the kernels directly.
 * A small two-dimensional FP64 problem (real data, n[0], n[1] <= 64, FP64
 * contraction, autonomous g) instead runs all nsteps steps in one fused
 * launch of a single workgroup with the state in LDS (expint_step then
 * launches it for one step); use_graph does not change the result.  Setting
 * the environment variable EXPINT_SMALL_FUSED=0 before expint_plan_create
 * keeps such a plan on the general kernel sequence.
 */
int expint_run(expint_plan* plan, void* U, double t0, int nsteps, int use_graph,
               void* ws, void* stream);

/* expint_plan_describe -- the launch configuration each mu-mode product (and
 * the launch of modes 1 and 2) of the plan's steps uses, one line per launch
 * shape: "family sizes: candidate (tuned, us)" or ": default".  Writes at most
 * len bytes including the terminating NUL into buf; *needed (optional) gets the
 * full length + 1.  Errors: EINVAL. */
int expint_plan_describe(const expint_plan* plan, char* buf, size_t len, size_t* needed);

/* expint_plan_is_fused -- *fused = 1 if the plan runs its steps in the fused
 * small-problem launch described at expint_run, else 0.  Errors: EINVAL. */
int expint_plan_is_fused(const expint_plan* plan, int* fused);

/*
 * expint_plan_check_finite -- whether the state U (device, the plan's layout and
 * element type) holds only finite values.  Enqueues one read of U on `stream`,
 * waits for the stream and returns EXPINT_OK, or EXPINT_ENONFINITE if an entry
 * (a real or imaginary part) is inf or nan.  Intended after expint_run /
 * expint_step, whose kernels do not test their results.  Uses one device int
 * of the plan: concurrent checks with the same plan race.
 * Errors: EINVAL (NULL plan or U, misaligned U), EHIP.
 */
int expint_plan_check_finite(expint_plan* plan, const void* U, void* stream);

/* expint_plan_destroy -- frees the plan's device memory and graph (NULL is a no-op).
 * The caller must make sure no enqueued work still uses the plan. */
void expint_plan_destroy(expint_plan* plan);

/* ------------------------------------------------------------------------ */
/* batched Riccati differential equations                                    */
/* ------------------------------------------------------------------------ */

typedef struct expint_batch_plan expint_batch_plan;

/*
 * expint_riccati_plan_create -- `count` independent instances of
 *     U' = A1 U + U A2^T + C + U B U,   U n1 x n2, B n2 x n1, C n1 x n2
 * (section 1, eq. Riccati; Kronecker form eq. ODE2d), each integrated with
 * ETD2RK phisplit (section 3.2; for d = 2 the phi_2 stage carries the split
 * factor 2).  phi_1 and phi_2 of tau A1 and tau A2 are built once on the host
 * in FP64.  A step is nine GEMM phases; each phase is one grouped launch
 * over all instances, each GEMM's tiles on one XCD, most expensive first.
 *   count   >= 1
 *   n1, n2  host arrays of count sizes, 1..4096
 *   A1, A2  host arrays of count host pointers, column-major n1 x n1 / n2 x n2 float64
 *   B, C    device float64, packed: instance i's B (column-major n2 x n1) and C
 *           (column-major n1 x n2) both start at element offset
 *           off_i = sum_{j<i} n1[j] n2[j].  They must stay valid while the plan is used.
 *   tau     step size
 * The state is one device array of sum n1 n2 float64 with instance i (column-major
 * n1 x n2) at off_i.  Errors: EINVAL, ENOTSUP, ENOMEM, EHIP.
 */
int expint_riccati_plan_create(expint_batch_plan** plan, int count, const int* n1, const int* n2,
                               const double* const* A1, const double* const* A2,
                               const double* B, const double* C, double tau);

/*
 * expint_riccati_plan_create_ex -- the same with a scheme: EXPINT_ETD2RK as
 * above, or EXPINT_ROSENBROCK_EULER (eq. expRosEulertensor, tau on the whole
 * bracket as in eq. expRosEuler).  The Jacobian of the right-hand side at U_n
 * is the Kronecker sum of J1 = A1 + U_n B and J2 = A2 + (B U_n)^T (the
 * structure section 4.1 states), and a step is
 *     U <- U + phi_1(tau J1) W phi_1(tau J2)^T,   W = tau (A1 U + U A2^T + C + U B U).
 * phi_1(tau J1) and phi_1(tau J2^T) = phi_1(tau J2)^T are built on the device
 * at every step in FP64: scaling by the even power of two that brings the
 * 1-norm to <= 1/2, the Taylor series of degree 13 by Horner (eq. seriesdef),
 * and the squaring recurrence eq. squarephi.  The number of squaring phases
 * per step is fixed at creation: the count ||tau A_mu||_1 needs plus 4.  A
 * Jacobian direction that needs more (its Taylor series would be evaluated
 * outside ||Y||_1 <= 1/2) is squared only that many times, and its step sets a
 * device flag that expint_batch_status reports as EXPINT_ENUMERIC.
 * Errors as expint_riccati_plan_create, and ENOTSUP for another scheme.
 */
int expint_riccati_plan_create_ex(expint_batch_plan** plan, int count, const int* n1, const int* n2,
                                  const double* const* A1, const double* const* A2, const double* B,
                                  const double* C, double tau, int scheme);

/* expint_batch_state_size -- elements of the packed state (sum n1 n2). */
int expint_batch_state_size(const expint_batch_plan* plan, size_t* elements);

/* expint_batch_workspace_size -- device workspace bytes of expint_batch_step/run. */
int expint_batch_workspace_size(const expint_batch_plan* plan, size_t* bytes);

/*
 * expint_batch_step / expint_batch_run -- one step / nsteps steps of every
 * instance, U (device, packed state) updated in place.  The first call with a
 * given (U, ws) pair builds and uploads the GEMM descriptors synchronously;
 * later calls with the same pair only enqueue.  use_graph != 0 replays one
 * captured step (needs a non-default stream).
 */
int expint_batch_step(expint_batch_plan* plan, double* U, void* ws, void* stream);
int expint_batch_run(expint_batch_plan* plan, double* U, int nsteps, int use_graph, void* ws, void* stream);

/*
 * expint_batch_tune -- the autotuner for the batched engine: each step is a
 * fixed sequence of grouped launches (one per phase), and each launch can put
 * its GEMMs on one tile class (64 x 64 or 128 x 64 outputs, with several K
 * chunk depths and occupancies) or on two classes in the same launch (128 x 64
 * outputs for the GEMMs with at least 128 rows, 64 x 64 for the rest).  This
 * times every grouped tile scheme on every phase, starting from one step of a
 * private copy of U (device, packed state, left unchanged; ws as for
 * expint_batch_step), and keeps the fastest per phase for the rest of the
 * process (and in EXPINT_TUNE_CACHE, as tucker_tune does).  Later steps of this
 * plan, and of plans with the same scheme and instance sizes, use the choice;
 * EXPINT_GROUPED (a scheme name) overrides it.  Every scheme computes the same
 * sums in the same order, so results do not depend on the choice.  The plan's
 * status words are restored.  Synchronous; allocates a copy of the state and
 * the descriptor lists, and frees them.  Errors: EINVAL (NULL or misaligned
 * arguments), ENOMEM, EHIP.
 */
int expint_batch_tune(expint_batch_plan* plan, double* U, void* ws, void* stream);

/*
 * expint_batch_describe -- one line per phase: "phase k: <scheme used> [<what
 * the autotuner holds for it>]".  Writes at most len bytes (NUL-terminated) to
 * buf (may be NULL) and the full size including the NUL to *needed (may be
 * NULL).  Errors: EINVAL (NULL plan), ENOMEM.
 */
int expint_batch_describe(const expint_batch_plan* plan, char* buf, size_t len, size_t* needed);

/*
 * expint_batch_status -- waits for `stream`, then reports what the steps
 * enqueued since the previous call found, and clears it:
 *   EXPINT_ENUMERIC   a Rosenbrock-Euler Jacobian direction needed more
 *                     squarings (section 3.1 scaling, eq. squarephi) than the
 *                     plan provides, so its phi_1 is inaccurate;
 *   EXPINT_ENONFINITE U (device packed state, optional: NULL skips the check)
 *                     holds inf or nan, or a Jacobian direction had a
 *                     non-finite 1-norm;
 *   EXPINT_OK         neither.
 * ENUMERIC is reported before ENONFINITE when both hold.  Synchronous.
 * Errors: EINVAL (NULL plan, misaligned U), EHIP.
 */
int expint_batch_status(expint_batch_plan* plan, const double* U, void* stream);

/* expint_batch_plan_destroy -- frees the plan (NULL is a no-op). */
void expint_batch_plan_destroy(expint_batch_plan* plan);

/* expint_last_error -- thread-local message of the last failing call ("" if none). */
const char* expint_last_error(void);

/* expint_version -- library version string. */
const char* expint_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EXPINT_H */
