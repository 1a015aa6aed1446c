// Batched Riccati differential equations, each integrated with ETD2RK phisplit.
//
// Instance i: U' = A1 U + U A2^T + C + U B U with U n1 x n2, B n2 x n1, C n1 x n2
// (paper section 1, eq. Riccati; Kronecker form eq. ODE2d with
// K = I (x) A1 + A2 (x) I, so K u = A1 U + U A2^T and a Tucker operator is
// M1 W M2^T).  One ETD2RK step (section 3.2, eq. ETD2RKtensor read with the
// split factor (2!)^{d-1} = 2 and tau on the whole first bracket) is nine
// GEMM phases; each phase is one grouped launch over all instances (each
// GEMM's tiles on one XCD, longest first):
//    1  T  = U B          (n1 <= n2)   or   B U   (n2 < n1),   and  W = tau U A2^T
//    2  Gn = C + T U                   or   C + U T
//    3  W  = tau A1 U + W + tau Gn
//    4  P  = phi1(tau A1) W
//    5  U2 = U + P phi1(tau A2)^T
//    6  T  = U2 B                      or   B U2
//    7  W2 = tau (T U2 + C - Gn)       or   tau (U2 T + C - Gn)
//    8  P  = phi2(tau A1) W2
//    9  U  = U2 + 2 P phi2(tau A2)^T
// (the two products of phase 1 depend on U alone; U A2^T reads the stored
// transpose of A2, so that every product of the phase has its B operand
// contiguous along k).
// The association of U B U is chosen per instance so the middle product is
// min(n1, n2) square.
//
// Exponential Rosenbrock-Euler (eq. expRosEulertensor, tau on the whole
// bracket as in eq. expRosEuler) needs phi_1 of the Jacobian directions at
// every step.  The Jacobian of f(U) = A1 U + U A2^T + C + U B U is the
// Kronecker sum with directions J1 = A1 + U B and J2 = A2 + (B U)^T (the
// structure section 4.1 states), and phi_1(tau J2)^T = phi_1(tau J2^T), so
// with X1 = tau J1 and X2 = tau J2^T = tau (A2^T + B U) one step is
//    U <- U + phi_1(X1) W phi_1(X2),   W = tau f(U) = tau A1 U + tau C + U X2
// (U X2 = tau U A2^T + tau U B U).  The phases:
//    R1  X1 = tau (A1 + U B),  X2 = tau (A2^T + B U)
//    R2  W  = tau A1 U + tau C               (one launch with R1: both read U alone)
//    R3  W  = W + U X2
//        k_phi_prep: s = the even power of two with ||X / 2^s||_1 <= 1/2,
//        Y = X / 2^s, H = Y / 14! + I / 13!
//    R4  twelve Horner steps H <- Y H + I / (k + 1)!  (k = 11 .. 0):
//        H = phi_1(Y) by its Taylor series to degree 13 (eq. seriesdef;
//        remainder below 2^-53 for ||Y||_1 <= 1/2)
//    R5  E = I + Y H = e^Y
//    R6  squarings (eq. squarephi): phi_1(2Y) = (phi_1(Y) e^Y + phi_1(Y)) / 2,
//        e^{2Y} = e^Y e^Y; a matrix takes part in squaring p while s > p
//    R7  P = phi_1(X1) W
//    R8  U = U + P phi_1(X2)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace expint;

namespace {

constexpr int kPhases = 9;  // ETD2RK
constexpr int kEtdDescs = 10;  // ETD2RK descriptors per instance and step (phase 1 has two)
constexpr int kHorner = 12;  // Rosenbrock-Euler: Horner GEMM steps after the prep kernel

// One matrix of the per-step phi_1 of the Rosenbrock-Euler scheme.
struct PhiJob {
  double* Y;  // in: X (n x n); out: X / 2^s
  double* H;  // out: Y / 14! + I / 13!
  int* s;     // out: the number of squarings (even, at most smax)
  int n;
};

// Device status words of a batched plan (cleared by expint_batch_status)
constexpr int kStatusSquarings = 0;  // a phi_1 needed more than smax squarings
constexpr int kStatusNonFinite = 1;  // a non-finite 1-norm or state

// One workgroup of 16 waves per matrix: the 1-norm (largest absolute column
// sum), the scaling, and the first Horner term.  Wave w takes columns w, w + 16,
// ...; lanes run down a column (coalesced).
constexpr int kPrepWaves = 16;
__global__ __launch_bounds__(64 * kPrepWaves) void k_phi_prep(const PhiJob* __restrict__ jobs, int smax,
                                                               int* __restrict__ status) {
  const PhiJob jb = jobs[blockIdx.x];
  const int n = jb.n, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double colmax[kPrepWaves];
  __shared__ int s_sh;
  double mx = 0.0;
  for (int c = wave; c < n; c += kPrepWaves) {
    const double* col = jb.Y + (long)n * c;
    double sum = 0.0;
    for (int i = lane; i < n; i += 64) sum += fabs(col[i]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
    mx = (sum > mx || sum != sum) ? sum : mx;
  }
  if (lane == 0) colmax[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double nu = colmax[0];
    for (int w = 1; w < kPrepWaves; ++w) nu = (colmax[w] > nu || colmax[w] != colmax[w]) ? colmax[w] : nu;
    int sc = 0;
    if (!(nu <= 1.7976931348623157e308)) {
      sc = smax;  // inf or nan: the result is not finite either way
      atomicOr(status + kStatusNonFinite, 1);
    } else {
      // the count that brings ||Y||_1 to <= 1/2 (at most 1100 halvings of a
      // finite norm); more than the plan's squaring phases is flagged and capped
      while (nu > 0.5) {
        nu *= 0.5;
        ++sc;
      }
      sc += sc & 1;  // even: the squarings end in the buffer they start from
      if (sc > smax) {
        atomicOr(status + kStatusSquarings, 1);
        sc = smax;
      }
    }
    s_sh = sc;
    *jb.s = sc;
  }
  __syncthreads();
  const double f = ldexp(1.0, -s_sh);
  const double c14 = 1.0 / 87178291200.0, c13 = 1.0 / 6227020800.0;  // 1/14!, 1/13!
  for (int c = wave; c < n; c += kPrepWaves) {
    double* ycol = jb.Y + (long)n * c;
    double* hcol = jb.H + (long)n * c;
    for (int i = lane; i < n; i += 64) {
      const double y = ycol[i] * f;
      ycol[i] = y;
      hcol[i] = y * c14 + (i == c ? c13 : 0.0);
    }
  }
}

// ETD2RK phases whose B operand is contiguous along k (the others read M^T, contiguous along q)
constexpr bool kPhaseBK[kPhases] = {true, true, true, true, false, true, true, true, false};

}  // namespace

struct expint_batch_plan {
  int count = 0;
  double tau = 0.0;
  std::vector<int> n1, n2;
  std::vector<long> uoff;     // state / B / C offsets (elements)
  std::vector<long> toff;     // T offsets
  std::vector<long> moff1;    // offsets of n1 x n1 matrices
  std::vector<long> moff2;    // offsets of n2 x n2 matrices
  std::vector<int> order;     // instances by decreasing cost
  long total = 0, ttotal = 0, m1total = 0, m2total = 0;
  const double* B = nullptr;  // caller's device arrays
  const double* C = nullptr;
  double* dA1 = nullptr;      // device copies: A1, phi1(tau A1), phi2(tau A1) (each m1total)
  double* dP1a = nullptr;
  double* dP2a = nullptr;
  double* dA2 = nullptr;      // A2, phi1(tau A2), phi2(tau A2) (each m2total)
  double* dP1b = nullptr;
  double* dP2b = nullptr;
  double* dA2T = nullptr;     // A2^T (m2total)
  int scheme = EXPINT_ETD2RK;
  int smax = 0;               // Rosenbrock-Euler: squaring phases per step
  std::vector<int> morder;    // Rosenbrock-Euler: the 2 count matrices by decreasing size
  // descriptors for the current (U, ws): one grouped launch per phase
  struct Phase {
    bool bk;                  // B operand contiguous along k
    long first;               // first descriptor
    int ndesc;
    long tiles;
    int scheme;               // grouped tile scheme (grouped_scheme_name)
    long map_off, blocks;     // its workgroup -> tile map (grouped_block_map)
  };
  std::vector<Phase> phases;
  int prep_after = -1;        // the phi prep kernel runs after this phase
  void* ddesc = nullptr;
  GroupedBlock* dmap = nullptr;
  PhiJob* djobs = nullptr;
  int* dstatus = nullptr;     // two status words (kStatus*)
  size_t desc_cap = 0, map_cap = 0;
  const void* d_U = nullptr;
  const void* d_ws = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace {

void free_batch(expint_batch_plan* p) {
  for (double* q : {p->dA1, p->dP1a, p->dP2a, p->dA2, p->dP1b, p->dP2b, p->dA2T})
    if (q) (void)hipFree(q);
  if (p->djobs) (void)hipFree(p->djobs);
  if (p->dstatus) (void)hipFree(p->dstatus);
  if (p->ddesc) (void)hipFree(p->ddesc);
  if (p->dmap) (void)hipFree(p->dmap);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
}

Epilogue linear(void* out, double alpha, const void* in1 = nullptr, double beta = 0.0, const void* in2 = nullptr,
                double c = 0.0) {
  Epilogue e;
  e.op = EPI_LINEAR;
  e.out0 = out;
  e.alpha = alpha;
  e.in1 = in1;
  e.beta = beta;
  e.in2 = in2;
  e.c = c;
  return e;
}

// The autotuner's key of phase k of a plan: the scheme, the number of squaring
// phases, the phase, and the instance sizes (count, total, and a hash of the list).
TuneKey grouped_key(const expint_batch_plan* p, int k) {
  unsigned long long h = 1469598103934665603ull;  // FNV-1a over the sizes
  for (int i = 0; i < p->count; ++i)
    for (int v : {p->n1[i], p->n2[i]}) {
      h ^= (unsigned)v;
      h *= 1099511628211ull;
    }
  const long a = (p->scheme == EXPINT_ROSENBROCK_EULER ? 1000000L : 0L) + 1000L * p->smax + k;
  return TuneKey{TUNE_GROUPED, a, p->count, p->total, (long)(h >> 2)};
}

// Descriptor lists of the phases, built on the host.  Phase k's tiles follow
// the grouped tile scheme `force` (>= 0), else the tuned choice of its key,
// else scheme 0.
struct PhaseBuilder {
  const expint_batch_plan* plan;
  int force;
  size_t dsz = gemm_desc_size();
  std::vector<char> desc;
  std::vector<GroupedBlock> map;
  std::vector<expint_batch_plan::Phase> phases;
  PhaseBuilder(const expint_batch_plan* p, int forced_scheme = -1) : plan(p), force(forced_scheme) {}
  char* open(bool bk) {  // a new phase
    expint_batch_plan::Phase ph;
    ph.bk = bk;
    ph.first = (long)(desc.size() / dsz);
    ph.ndesc = 0;
    ph.tiles = 0;
    ph.map_off = 0;
    ph.blocks = 0;
    ph.scheme = force >= 0 ? force : std::max(0, tune_choice(grouped_key(plan, (int)phases.size())));
    phases.push_back(ph);
    return nullptr;
  }
  char* add() {  // room for one more descriptor of the open phase
    desc.resize(desc.size() + dsz);
    return desc.data() + desc.size() - dsz;
  }
  void added() {  // after make_gemm_desc filled the last descriptor
    auto& ph = phases.back();
    char* d = desc.data() + desc.size() - dsz;
    gemm_desc_set_scheme(d, ph.scheme);
    ph.tiles += gemm_desc_tiles(d);
    ph.ndesc += 1;
  }
  bool finish() {  // every phase's workgroup map, after the last descriptor
    std::vector<GroupedBlock> m;
    for (auto& ph : phases) {
      grouped_block_map(desc.data() + (size_t)ph.first * dsz, ph.ndesc, ph.scheme, m);
      if (!grouped_block_map_valid(desc.data() + (size_t)ph.first * dsz, ph.ndesc, m)) return false;
      ph.map_off = (long)map.size();
      ph.blocks = (long)m.size();
      map.insert(map.end(), m.begin(), m.end());
    }
    return true;
  }
};

// ETD2RK: the nine phases listed at the top of this file.
void build_etd2rk(expint_batch_plan* p, double* U, char* ws, PhaseBuilder& pb) {
  const int cnt = p->count;
  double* T = reinterpret_cast<double*>(ws);
  double* Gn = T + p->ttotal;
  double* W = Gn + p->total;
  double* P = W + p->total;
  double* U2 = P + p->total;
  double* W2 = U2 + p->total;
  const double tau = p->tau;
  for (int ph = 0; ph < kPhases; ++ph) {
    pb.open(kPhaseBK[ph]);
    for (int slot = 0; slot < cnt; ++slot) {
      const int i = p->order[slot];
      const long n1 = p->n1[i], n2 = p->n2[i];
      const long uo = p->uoff[i], to = p->toff[i];
      const bool left = n1 <= n2;  // T = U B (n1 x n1) else T = B U (n2 x n2)
      double* Ui = U + uo;
      double* U2i = U2 + uo;
      const double* Bi = p->B + uo;
      const double* Ci = p->C + uo;
      double* Ti = T + to;
      double *Gi = Gn + uo, *Wi = W + uo, *Pi = P + uo, *W2i = W2 + uo;
      const double *A1 = p->dA1 + p->moff1[i], *P1a = p->dP1a + p->moff1[i], *P2a = p->dP2a + p->moff1[i];
      const double *A2T = p->dA2T + p->moff2[i], *P1b = p->dP1b + p->moff2[i], *P2b = p->dP2b + p->moff2[i];
      switch (ph) {
        case 0:  // T = U B  or  B U;  W = tau U A2^T  (B operand A2^T[k, q] = A2T[k + n2 q])
          if (left)
            make_gemm_desc(pb.add(), Ui, n1, Bi, 1, n2, n1, n1, n2, n1, linear(Ti, 1.0));
          else
            make_gemm_desc(pb.add(), Bi, n2, Ui, 1, n1, n2, n2, n1, n2, linear(Ti, 1.0));
          pb.added();
          make_gemm_desc(pb.add(), Ui, n1, A2T, 1, n2, n1, n2, n2, n1, linear(Wi, tau));
          break;
        case 5:  // T = U2 B  or  B U2
          if (left)
            make_gemm_desc(pb.add(), U2i, n1, Bi, 1, n2, n1, n1, n2, n1, linear(Ti, 1.0));
          else
            make_gemm_desc(pb.add(), Bi, n2, U2i, 1, n1, n2, n2, n1, n2, linear(Ti, 1.0));
          break;
        case 1:  // Gn = C + T U  or  C + U T
          if (left)
            make_gemm_desc(pb.add(), Ti, n1, Ui, 1, n1, n1, n2, n1, n1, linear(Gi, 1.0, Ci, 1.0));
          else
            make_gemm_desc(pb.add(), Ui, n1, Ti, 1, n2, n1, n2, n2, n1, linear(Gi, 1.0, Ci, 1.0));
          break;
        case 6:  // W2 = tau (T U2 + C - Gn)  or  tau (U2 T + C - Gn)
          if (left)
            make_gemm_desc(pb.add(), Ti, n1, U2i, 1, n1, n1, n2, n1, n1, linear(W2i, tau, Ci, tau, Gi, -tau));
          else
            make_gemm_desc(pb.add(), U2i, n1, Ti, 1, n2, n1, n2, n2, n1, linear(W2i, tau, Ci, tau, Gi, -tau));
          break;
        case 2:  // W = tau A1 U + W + tau Gn
          make_gemm_desc(pb.add(), A1, n1, Ui, 1, n1, n1, n2, n1, n1, linear(Wi, tau, Wi, 1.0, Gi, tau));
          break;
        case 3:  // P = phi1(tau A1) W
          make_gemm_desc(pb.add(), P1a, n1, Wi, 1, n1, n1, n2, n1, n1, linear(Pi, 1.0));
          break;
        case 4:  // U2 = U + P phi1(tau A2)^T
          make_gemm_desc(pb.add(), Pi, n1, P1b, n2, 1, n1, n2, n2, n1, linear(U2i, 1.0, Ui, 1.0));
          break;
        case 7:  // P = phi2(tau A1) W2
          make_gemm_desc(pb.add(), P2a, n1, W2i, 1, n1, n1, n2, n1, n1, linear(Pi, 1.0));
          break;
        case 8:  // U = U2 + 2 P phi2(tau A2)^T
          make_gemm_desc(pb.add(), Pi, n1, P2b, n2, 1, n1, n2, n2, n1, linear(Ui, 2.0, U2i, 1.0));
          break;
      }
      pb.added();
    }
  }
}

// Rosenbrock-Euler: the phases R1 .. R8 listed at the top of this file.
void build_rosenbrock(expint_batch_plan* p, double* U, char* ws, PhaseBuilder& pb, std::vector<PhiJob>& jobs) {
  const int cnt = p->count;
  const double tau = p->tau;
  double* W = reinterpret_cast<double*>(ws);
  double* P = W + p->total;
  double* m1 = P + p->total;         // Y, Ha, Hb, Ea, Eb of direction 1 (each m1total)
  double* m2 = m1 + 5 * p->m1total;  // the same for direction 2 (each m2total)
  int* sc = reinterpret_cast<int*>(m2 + 5 * p->m2total);  // 2 count squaring counts
  // matrix j < cnt: direction 1 of instance j; j >= cnt: direction 2 of instance j - cnt
  auto mat = [&](int j, int which) -> double* {  // which: 0 Y, 1 Ha, 2 Hb, 3 Ea, 4 Eb
    if (j < cnt) return m1 + which * p->m1total + p->moff1[j];
    return m2 + which * p->m2total + p->moff2[j - cnt];
  };
  auto msize = [&](int j) -> long { return j < cnt ? p->n1[j] : p->n2[j - cnt]; };
  // R1: X1 = tau (A1 + U B), X2 = tau (A2^T + B U)
  pb.open(true);
  for (int slot = 0; slot < cnt; ++slot) {
    const int i = p->order[slot];
    const long n1 = p->n1[i], n2 = p->n2[i], uo = p->uoff[i];
    make_gemm_desc(pb.add(), U + uo, n1, p->B + uo, 1, n2, n1, n1, n2, n1,
                   linear(mat(i, 0), tau, p->dA1 + p->moff1[i], tau));
    pb.added();
    make_gemm_desc(pb.add(), p->B + uo, n2, U + uo, 1, n1, n2, n2, n1, n2,
                   linear(mat(cnt + i, 0), tau, p->dA2T + p->moff2[i], tau));
    pb.added();
  }
  // R2: W = tau A1 U + tau C (in the launch of R1: both read U alone)
  for (int slot = 0; slot < cnt; ++slot) {
    const int i = p->order[slot];
    const long n1 = p->n1[i], n2 = p->n2[i], uo = p->uoff[i];
    make_gemm_desc(pb.add(), p->dA1 + p->moff1[i], n1, U + uo, 1, n1, n1, n2, n1, n1,
                   linear(W + uo, tau, p->C + uo, tau));
    pb.added();
  }
  // R3: W = W + U X2
  pb.open(true);
  for (int slot = 0; slot < cnt; ++slot) {
    const int i = p->order[slot];
    const long n1 = p->n1[i], n2 = p->n2[i], uo = p->uoff[i];
    make_gemm_desc(pb.add(), U + uo, n1, mat(cnt + i, 0), 1, n2, n1, n2, n2, n1, linear(W + uo, 1.0, W + uo, 1.0));
    pb.added();
  }
  // the prep kernel follows R3
  jobs.clear();
  for (int j : p->morder) jobs.push_back(PhiJob{mat(j, 0), mat(j, 1), sc + j, (int)msize(j)});
  auto diag = [](double* out, double c, long n) {
    Epilogue e;
    e.op = EPI_DIAG;
    e.out0 = out;
    e.alpha = 1.0;
    e.c = c;
    e.ldiag = n + 1;
    return e;
  };
  // R4: Horner steps H <- Y H + I / (k + 1)!, k = 11 .. 0 (Ha -> Hb -> Ha ...)
  double fact = 1.0;
  std::vector<double> inv_fact(14);
  for (int k = 0; k < 14; ++k) {
    fact *= (k + 1);
    inv_fact[k] = 1.0 / fact;  // 1 / (k + 1)!
  }
  for (int step = 0; step < kHorner; ++step) {
    const int k = kHorner - 1 - step;
    const int src = (step % 2 == 0) ? 1 : 2, dst = 3 - src;
    pb.open(true);
    for (int j : p->morder) {
      const long n = msize(j);
      make_gemm_desc(pb.add(), mat(j, 0), n, mat(j, src), 1, n, n, n, n, n, diag(mat(j, dst), inv_fact[k], n));
      pb.added();
    }
  }
  // R5: Ea = I + Y Ha
  pb.open(true);
  for (int j : p->morder) {
    const long n = msize(j);
    make_gemm_desc(pb.add(), mat(j, 0), n, mat(j, 1), 1, n, n, n, n, n, diag(mat(j, 3), 1.0, n));
    pb.added();
  }
  // R6: squarings, gated by each matrix's count
  for (int q = 0; q < p->smax; ++q) {
    const int hc = (q % 2 == 0) ? 1 : 2, hn = 3 - hc;
    const int ec = (q % 2 == 0) ? 3 : 4, en = 7 - ec;
    pb.open(true);
    for (int j : p->morder) {
      const long n = msize(j);
      make_gemm_desc(pb.add(), mat(j, hc), n, mat(j, ec), 1, n, n, n, n, n, linear(mat(j, hn), 0.5, mat(j, hc), 0.5),
                     sc + j, q);
      pb.added();
      make_gemm_desc(pb.add(), mat(j, ec), n, mat(j, ec), 1, n, n, n, n, n, linear(mat(j, en), 1.0), sc + j, q);
      pb.added();
    }
  }
  // R7: P = phi_1(X1) W;  R8: U = U + P phi_1(X2)
  pb.open(true);
  for (int slot = 0; slot < cnt; ++slot) {
    const int i = p->order[slot];
    const long n1 = p->n1[i], n2 = p->n2[i], uo = p->uoff[i];
    make_gemm_desc(pb.add(), mat(i, 1), n1, W + uo, 1, n1, n1, n2, n1, n1, linear(P + uo, 1.0));
    pb.added();
  }
  pb.open(true);
  for (int slot = 0; slot < cnt; ++slot) {
    const int i = p->order[slot];
    const long n1 = p->n1[i], n2 = p->n2[i], uo = p->uoff[i];
    make_gemm_desc(pb.add(), P + uo, n1, mat(cnt + i, 1), 1, n2, n1, n2, n2, n1, linear(U + uo, 1.0, U + uo, 1.0));
    pb.added();
  }
}

int build_phases(expint_batch_plan* p, double* U, char* ws, PhaseBuilder& pb, std::vector<PhiJob>& jobs) {
  if (p->scheme == EXPINT_ROSENBROCK_EULER) {
    build_rosenbrock(p, U, ws, pb, jobs);
    p->prep_after = 1;
  } else {
    build_etd2rk(p, U, ws, pb);
    p->prep_after = -1;
  }
  if (!pb.finish()) return set_error(EXPINT_EINVAL, "internal error: a grouped workgroup map misses or repeats a tile");
  return EXPINT_OK;
}

// Build every phase's descriptors for state U and workspace ws and upload them.
int build_descriptors(expint_batch_plan* p, double* U, char* ws) {
  PhaseBuilder pb(p);
  std::vector<PhiJob> jobs;
  if (const int rc = build_phases(p, U, ws, pb, jobs); rc != EXPINT_OK) return rc;
  // descriptors of an earlier (U, ws) pair may still be read by enqueued work
  if (p->d_U && hipDeviceSynchronize() != hipSuccess)
    return set_error(EXPINT_EHIP, "device synchronisation before a descriptor rebuild failed");
  if (pb.desc.size() > p->desc_cap) return set_error(EXPINT_EINVAL, "batched descriptors exceed the plan's capacity");
  if (pb.map.size() > p->map_cap) {  // the maps' size depends on the tuned tile schemes
    if (p->dmap) (void)hipFree(p->dmap);
    p->dmap = nullptr;
    p->map_cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(&p->dmap), pb.map.size() * sizeof(GroupedBlock)) != hipSuccess)
      return set_error(EXPINT_ENOMEM, "device allocation for the workgroup maps failed");
    p->map_cap = pb.map.size();
  }
  if (hipMemcpy(p->ddesc, pb.desc.data(), pb.desc.size(), hipMemcpyHostToDevice) != hipSuccess ||
      (!pb.map.empty() && hipMemcpy(p->dmap, pb.map.data(), pb.map.size() * sizeof(GroupedBlock),
                                    hipMemcpyHostToDevice) != hipSuccess) ||
      (!jobs.empty() &&
       hipMemcpy(p->djobs, jobs.data(), jobs.size() * sizeof(PhiJob), hipMemcpyHostToDevice) != hipSuccess))
    return set_error(EXPINT_EHIP, "upload of batched GEMM descriptors failed");
  p->phases = pb.phases;
  p->d_U = U;
  p->d_ws = ws;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return EXPINT_OK;
}

int enqueue_batch_step(expint_batch_plan* p, hipStream_t s) {
  const size_t dsz = gemm_desc_size();
  for (size_t k = 0; k < p->phases.size(); ++k) {
    const auto& ph = p->phases[k];
    const char* d = static_cast<const char*>(p->ddesc) + (size_t)ph.first * dsz;
    const int rc = launch_grouped_gemm(ph.bk, d, p->dmap + ph.map_off, ph.blocks, ph.scheme, s);
    if (rc != EXPINT_OK) return rc;
    if ((int)k == p->prep_after) {
      hipLaunchKernelGGL(k_phi_prep, dim3(2 * p->count), dim3(64 * kPrepWaves), 0, s, p->djobs, p->smax,
                         p->dstatus);
      const hipError_t err = hipGetLastError();
      if (err != hipSuccess) return set_error(EXPINT_EHIP, "phi prep launch failed: %s", hipGetErrorString(err));
    }
  }
  return EXPINT_OK;
}

int prepare(expint_batch_plan* p, double* U, void* ws) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  if (!U || !ws) return set_error(EXPINT_EINVAL, "U and ws must be non-NULL device pointers");
  if ((reinterpret_cast<uintptr_t>(U) & 15u) || (reinterpret_cast<uintptr_t>(ws) & 15u))
    return set_error(EXPINT_EINVAL, "U and ws must be 16-byte aligned");
  if (p->d_U != U || p->d_ws != ws) {
    try {  // host vectors and the tuning table: nothing may throw across the C ABI
      return build_descriptors(p, U, static_cast<char*>(ws));
    } catch (...) {
      return set_error(EXPINT_ENOMEM, "host resources exhausted while building the batched descriptors");
    }
  }
  return EXPINT_OK;
}

}  // namespace

namespace {

// Frees a partly built plan when creation returns early or a host allocation throws.
struct BatchPlanGuard {
  expint_batch_plan* p = nullptr;
  ~BatchPlanGuard() {
    if (p) {
      free_batch(p);
      delete p;
    }
  }
};

int riccati_plan_create(expint_batch_plan** out, int count, const int* n1, const int* n2, const double* const* A1,
                        const double* const* A2, const double* B, const double* C, double tau, int scheme) {
  if (scheme != EXPINT_ETD2RK && scheme != EXPINT_ROSENBROCK_EULER)
    return set_error(EXPINT_ENOTSUP, "batched Riccati plans support ETD2RK and Rosenbrock-Euler (scheme %d)", scheme);
  const bool ros = scheme == EXPINT_ROSENBROCK_EULER;
  if (count < 1 || !n1 || !n2 || !A1 || !A2 || !B || !C)
    return set_error(EXPINT_EINVAL, "need count >= 1 and non-NULL size, matrix and B/C arrays");
  if (!std::isfinite(tau)) return set_error(EXPINT_EINVAL, "tau is not finite");
  long total = 0;
  for (int i = 0; i < count; ++i) {
    if (n1[i] < 1 || n2[i] < 1) return set_error(EXPINT_EINVAL, "instance %d: sizes must be >= 1", i);
    if (n1[i] > 4096 || n2[i] > 4096) return set_error(EXPINT_ENOTSUP, "instance %d: sizes above 4096", i);
    if (!A1[i] || !A2[i]) return set_error(EXPINT_EINVAL, "instance %d: NULL A1 or A2", i);
    total += (long)n1[i] * n2[i];
  }
  if (total * 8 >= (1L << 31)) return set_error(EXPINT_ENOTSUP, "batched state above 2 GiB");
  BatchPlanGuard guard;
  expint_batch_plan* p = guard.p = new (std::nothrow) expint_batch_plan();
  if (!p) return set_error(EXPINT_ENOMEM, "plan allocation failed");
  p->count = count;
  p->tau = tau;
  p->scheme = scheme;
  p->B = B;
  p->C = C;
  p->n1.assign(n1, n1 + count);
  p->n2.assign(n2, n2 + count);
  p->uoff.resize(count);
  p->toff.resize(count);
  p->moff1.resize(count);
  p->moff2.resize(count);
  for (int i = 0; i < count; ++i) {
    p->uoff[i] = p->total;
    p->toff[i] = p->ttotal;
    p->moff1[i] = p->m1total;
    p->moff2[i] = p->m2total;
    const long m = std::min(n1[i], n2[i]);
    p->total += (long)n1[i] * n2[i];
    p->ttotal += m * m;
    p->m1total += (long)n1[i] * n1[i];
    p->m2total += (long)n2[i] * n2[i];
  }
  p->order.resize(count);
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) {
    const double ca = (double)n1[a] * n2[a] * (n1[a] + n2[a]), cb = (double)n1[b] * n2[b] * (n1[b] + n2[b]);
    return ca > cb;
  });
  // phi_1 and phi_2 of tau A1_i and tau A2_i on the host, FP64 (once per run)
  std::vector<double> hA1(p->m1total), hP1a(p->m1total), hP2a(p->m1total);
  std::vector<double> hA2(p->m2total), hP1b(p->m2total), hP2b(p->m2total);
  std::vector<int> rcs(2 * count, EXPINT_OK);
  auto work_job = [&](int job) {
    const int i = job / 2;
    const bool first = (job % 2) == 0;
    const int n = first ? n1[i] : n2[i];
    const double* A = first ? A1[i] : A2[i];
    double* dstA = (first ? hA1.data() + p->moff1[i] : hA2.data() + p->moff2[i]);
    std::memcpy(dstA, A, sizeof(double) * n * n);
    if (ros) return;  // phi of the Jacobian directions is built on the device at every step
    std::vector<double> buf((size_t)3 * n * n);
    phi_setup_single_threaded(true);  // the jobs already run in parallel
    rcs[job] = phi_setup_real(n, A, n, tau, 2, buf.data(), n);
    double* dst1 = (first ? hP1a.data() + p->moff1[i] : hP1b.data() + p->moff2[i]);
    double* dst2 = (first ? hP2a.data() + p->moff1[i] : hP2b.data() + p->moff2[i]);
    std::memcpy(dst1, buf.data() + (size_t)n * n, sizeof(double) * n * n);
    std::memcpy(dst2, buf.data() + (size_t)2 * n * n, sizeof(double) * n * n);
  };
  // a failure inside a job (host allocation) marks that job; no exception leaves a thread
  auto work = [&](int job) noexcept {
    try {
      work_job(job);
    } catch (...) {
      rcs[job] = EXPINT_ENOMEM;
    }
  };
  {
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    std::vector<std::thread> pool;
    std::atomic<int> next{0};
    auto drain = [&]() noexcept {
      for (int job = next++; job < 2 * count; job = next++) work(job);
    };
    try {
      pool.reserve(nt);
      for (unsigned t = 1; t < nt; ++t) pool.emplace_back(drain);
    } catch (...) {
      // fewer threads: the calling thread takes the remaining jobs below
    }
    drain();
    phi_setup_single_threaded(false);  // the calling thread's later phi_setup calls may use threads again
    for (auto& th : pool) th.join();
  }
  int rc = EXPINT_OK;
  for (int job = 0; job < 2 * count && rc == EXPINT_OK; ++job)
    if (rcs[job] != EXPINT_OK)
      rc = set_error(rcs[job], "phi setup of instance %d (direction %d) failed (status %d)", job / 2, job % 2 + 1,
                     rcs[job]);
  auto upload = [&](double** dst, const std::vector<double>& src) {
    if (rc != EXPINT_OK) return;
    if (hipMalloc(dst, src.size() * sizeof(double)) != hipSuccess) {
      rc = set_error(EXPINT_ENOMEM, "device allocation failed");
      return;
    }
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      rc = set_error(EXPINT_EHIP, "upload failed");
  };
  upload(&p->dA1, hA1);
  upload(&p->dA2, hA2);
  {
    // A2^T (column-major n2 x n2 per instance): the B operand of U A2^T contiguous along k
    std::vector<double> hA2T(p->m2total);
    for (int i = 0; i < count; ++i) {
      const long m = n2[i];
      for (long r = 0; r < m; ++r)
        for (long c = 0; c < m; ++c) hA2T[p->moff2[i] + r + m * c] = A2[i][c + m * r];
    }
    upload(&p->dA2T, hA2T);
  }
  size_t ndesc = 0;
  if (!ros) {
    upload(&p->dP1a, hP1a);
    upload(&p->dP2a, hP2a);
    upload(&p->dP1b, hP1b);
    upload(&p->dP2b, hP2b);
    ndesc = (size_t)kEtdDescs * count;
  } else {
    // the matrices by decreasing size, and the number of squaring phases: the
    // largest count ||tau A_mu||_1 needs, plus 4 for the U B terms of the
    // Jacobian (a matrix needing more is squared that many times only)
    double numax = 0.0;
    for (int i = 0; i < count; ++i) {
      for (int dir = 0; dir < 2; ++dir) {
        const long n = dir ? n2[i] : n1[i];
        const double* A = dir ? A2[i] : A1[i];
        for (long c = 0; c < n; ++c) {
          double sum = 0.0;
          for (long r = 0; r < n; ++r) sum += std::fabs(A[r + n * c]);
          numax = std::max(numax, std::fabs(tau) * sum);
        }
      }
    }
    int sc = 0;
    while (numax > 0.5 && sc < 60) {
      numax *= 0.5;
      ++sc;
    }
    p->smax = sc + 4 + ((sc + 4) & 1);
    p->morder.resize(2 * count);
    std::iota(p->morder.begin(), p->morder.end(), 0);
    std::stable_sort(p->morder.begin(), p->morder.end(), [&](int a, int b) {
      const int na = a < count ? n1[a] : n2[a - count], nb = b < count ? n1[b] : n2[b - count];
      return na > nb;
    });
    ndesc = (size_t)count * (32 + 4 * p->smax);
    if (rc == EXPINT_OK && hipMalloc(reinterpret_cast<void**>(&p->djobs), 2 * count * sizeof(PhiJob)) != hipSuccess)
      rc = set_error(EXPINT_ENOMEM, "device allocation for phi jobs failed");
  }
  p->desc_cap = ndesc * gemm_desc_size();
  if (rc == EXPINT_OK && hipMalloc(&p->ddesc, p->desc_cap) != hipSuccess)
    rc = set_error(EXPINT_ENOMEM, "device allocation for descriptors failed");
  if (rc == EXPINT_OK) {
    if (hipMalloc(reinterpret_cast<void**>(&p->dstatus), 2 * sizeof(int)) != hipSuccess)
      rc = set_error(EXPINT_ENOMEM, "device allocation for the status words failed");
    else if (hipMemset(p->dstatus, 0, 2 * sizeof(int)) != hipSuccess)
      rc = set_error(EXPINT_EHIP, "status word initialisation failed");
  }
  if (rc != EXPINT_OK) return rc;
  guard.p = nullptr;
  *out = p;
  return EXPINT_OK;
}

}  // namespace

extern "C" int expint_riccati_plan_create_ex(expint_batch_plan** out, int count, const int* n1, const int* n2,
                                             const double* const* A1, const double* const* A2, const double* B,
                                             const double* C, double tau, int scheme) {
  if (!out) return set_error(EXPINT_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  try {
    return riccati_plan_create(out, count, n1, n2, A1, A2, B, C, tau, scheme);
  } catch (const std::bad_alloc&) {
    return set_error(EXPINT_ENOMEM, "host allocation failed while creating the batched plan");
  } catch (...) {
    return set_error(EXPINT_ENOMEM, "host resources exhausted while creating the batched plan");
  }
}

extern "C" int expint_riccati_plan_create(expint_batch_plan** out, int count, const int* n1, const int* n2,
                                          const double* const* A1, const double* const* A2, const double* B,
                                          const double* C, double tau) {
  return expint_riccati_plan_create_ex(out, count, n1, n2, A1, A2, B, C, tau, EXPINT_ETD2RK);
}

extern "C" int expint_batch_state_size(const expint_batch_plan* p, size_t* elements) {
  if (!p || !elements) return set_error(EXPINT_EINVAL, "NULL plan or output");
  *elements = (size_t)p->total;
  return EXPINT_OK;
}

extern "C" int expint_batch_workspace_size(const expint_batch_plan* p, size_t* bytes) {
  if (!p || !bytes) return set_error(EXPINT_EINVAL, "NULL plan or output");
  if (p->scheme == EXPINT_ROSENBROCK_EULER)
    *bytes = (size_t)(2 * p->total + 5 * (p->m1total + p->m2total)) * sizeof(double) + 2 * p->count * sizeof(int);
  else
    *bytes = (size_t)(p->ttotal + 5 * p->total) * sizeof(double);
  return EXPINT_OK;
}

extern "C" int expint_batch_step(expint_batch_plan* p, double* U, void* ws, void* stream) {
  const int rc = prepare(p, U, ws);
  if (rc != EXPINT_OK) return rc;
  return enqueue_batch_step(p, static_cast<hipStream_t>(stream));
}

extern "C" int expint_batch_run(expint_batch_plan* p, double* U, int nsteps, int use_graph, void* ws,
                                void* stream) {
  int rc = prepare(p, U, ws);
  if (rc != EXPINT_OK) return rc;
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!use_graph) {
    for (int k = 0; k < nsteps; ++k)
      if ((rc = enqueue_batch_step(p, s)) != EXPINT_OK) return rc;
    return EXPINT_OK;
  }
  if (!s) return set_error(EXPINT_EINVAL, "graph capture needs a non-default stream");
  if (!p->gexec || p->g_stream != s) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(EXPINT_EHIP, "stream capture could not start");
    rc = enqueue_batch_step(p, s);
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != EXPINT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess) return set_error(EXPINT_EHIP, "stream capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      p->gexec = nullptr;
      return set_error(EXPINT_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    p->g_stream = s;
  }
  for (int k = 0; k < nsteps; ++k)
    if (hipGraphLaunch(p->gexec, s) != hipSuccess) return set_error(EXPINT_EHIP, "graph launch failed");
  return EXPINT_OK;
}

extern "C" int expint_batch_status(expint_batch_plan* p, const double* U, void* stream) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  if (U && (reinterpret_cast<uintptr_t>(U) & 15u)) return set_error(EXPINT_EINVAL, "U must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (U) {
    const int rc = launch_finite_check(U, p->total, p->dstatus + kStatusNonFinite, s);
    if (rc != EXPINT_OK) return rc;
  }
  int st[2] = {0, 0};
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(st, p->dstatus, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(EXPINT_EHIP, "reading the batched plan's status failed");
  if (st[0] || st[1]) {
    if (hipMemset(p->dstatus, 0, sizeof(st)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
      return set_error(EXPINT_EHIP, "clearing the batched plan's status failed");
  }
  if (st[kStatusSquarings])
    return set_error(EXPINT_ENUMERIC, "a Jacobian direction needed more than the plan's %d squarings: its phi_1 is "
                     "inaccurate", p->smax);
  if (st[kStatusNonFinite]) return set_error(EXPINT_ENONFINITE, "the state or a Jacobian direction is not finite");
  return EXPINT_OK;
}

namespace {

// Times every grouped tile scheme on every phase of the plan and keeps the
// fastest per phase (the autotuner's table; EXPINT_TUNE_CACHE keeps it across
// processes).  The steps run on a private copy of U in ws; the caller's U and
// the plan's status words are left as they were.
int batch_tune(expint_batch_plan* p, double* U, char* ws, hipStream_t s) {
  const int ns = grouped_scheme_count();
  const size_t dsz = gemm_desc_size();
  double* tU = nullptr;
  std::vector<void*> dd(ns, nullptr);
  std::vector<GroupedBlock*> dmp(ns, nullptr);
  std::vector<std::vector<expint_batch_plan::Phase>> ph(ns);
  int saved[2] = {0, 0};
  int rc = EXPINT_OK;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(saved, p->dstatus, sizeof(saved), hipMemcpyDeviceToHost) != hipSuccess)
    rc = set_error(EXPINT_EHIP, "batch tuning: reading the status words failed");
  if (rc == EXPINT_OK && hipMalloc(reinterpret_cast<void**>(&tU), p->total * sizeof(double)) != hipSuccess)
    rc = set_error(EXPINT_ENOMEM, "batch tuning: state copy allocation failed");
  if (rc == EXPINT_OK &&
      hipMemcpyAsync(tU, U, p->total * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
    rc = set_error(EXPINT_EHIP, "batch tuning: state copy failed");
  // every scheme's descriptors for the copy (scheme 0 also becomes the plan's current set)
  std::vector<PhiJob> jobs;
  for (int c = 0; c < ns && rc == EXPINT_OK; ++c) {
    PhaseBuilder pb(p, c);
    jobs.clear();
    if ((rc = build_phases(p, tU, ws, pb, jobs)) != EXPINT_OK) break;
    ph[c] = pb.phases;
    if (hipMalloc(&dd[c], pb.desc.size()) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&dmp[c]), std::max<size_t>(1, pb.map.size()) * sizeof(GroupedBlock)) !=
            hipSuccess) {
      rc = set_error(EXPINT_ENOMEM, "batch tuning: descriptor allocation failed");
      break;
    }
    if (hipMemcpy(dd[c], pb.desc.data(), pb.desc.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (!pb.map.empty() && hipMemcpy(dmp[c], pb.map.data(), pb.map.size() * sizeof(GroupedBlock),
                                      hipMemcpyHostToDevice) != hipSuccess) ||
        (!jobs.empty() && c == 0 &&
         hipMemcpy(p->djobs, jobs.data(), jobs.size() * sizeof(PhiJob), hipMemcpyHostToDevice) != hipSuccess))
      rc = set_error(EXPINT_EHIP, "batch tuning: descriptor upload failed");
  }
  auto launch_phase = [&](int c, int k) {
    const auto& q = ph[c][k];
    return launch_grouped_gemm(q.bk, static_cast<const char*>(dd[c]) + (size_t)q.first * dsz,
                               dmp[c] + q.map_off, q.blocks, q.scheme, s);
  };
  // one whole step first, so that the workspace and the squaring counts hold a step's values
  const int nph = rc == EXPINT_OK ? (int)ph[0].size() : 0;
  for (int k = 0; k < nph && rc == EXPINT_OK; ++k) {
    rc = launch_phase(0, k);
    if (rc == EXPINT_OK && k == p->prep_after) {
      hipLaunchKernelGGL(k_phi_prep, dim3(2 * p->count), dim3(64 * kPrepWaves), 0, s, p->djobs, p->smax,
                         p->dstatus);
      if (hipGetLastError() != hipSuccess) rc = set_error(EXPINT_EHIP, "batch tuning: phi prep launch failed");
    }
  }
  for (int k = 0; k < nph && rc == EXPINT_OK; ++k) {
    const TuneKey key = grouped_key(p, k);
    rc = tune_key(key, s, [&]() { return launch_phase(std::max(0, tune_choice(key)), k); });
  }
  if (hipStreamSynchronize(s) != hipSuccess && rc == EXPINT_OK)
    rc = set_error(EXPINT_EHIP, "batch tuning: synchronisation failed");
  if (hipMemcpy(p->dstatus, saved, sizeof(saved), hipMemcpyHostToDevice) != hipSuccess && rc == EXPINT_OK)
    rc = set_error(EXPINT_EHIP, "batch tuning: restoring the status words failed");
  if (tU) (void)hipFree(tU);
  for (int c = 0; c < ns; ++c) {
    if (dd[c]) (void)hipFree(dd[c]);
    if (dmp[c]) (void)hipFree(dmp[c]);
  }
  // the next step rebuilds the descriptors (and the graph) with the tuned schemes
  p->d_U = nullptr;
  p->d_ws = nullptr;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return rc;
}

}  // namespace

extern "C" int expint_batch_tune(expint_batch_plan* p, double* U, void* ws, void* stream) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  if (!U || !ws) return set_error(EXPINT_EINVAL, "U and ws must be non-NULL device pointers");
  if ((reinterpret_cast<uintptr_t>(U) & 15u) || (reinterpret_cast<uintptr_t>(ws) & 15u))
    return set_error(EXPINT_EINVAL, "U and ws must be 16-byte aligned");
  try {
    return batch_tune(p, U, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  } catch (...) {
    return set_error(EXPINT_ENOMEM, "host resources exhausted while tuning the batched plan");
  }
}

extern "C" int expint_batch_describe(const expint_batch_plan* p, char* buf, size_t len, size_t* needed) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  std::string text;
  try {
    const int nph = p->scheme == EXPINT_ROSENBROCK_EULER ? 17 + p->smax : kPhases;
    for (int k = 0; k < nph; ++k) {
      const TuneKey key = grouped_key(p, k);
      const int c = tune_choice(key);
      text += "phase " + std::to_string(k + 1) + ": " + grouped_scheme_name(std::max(0, c)) + " [" +
              tune_describe(key) + "]\n";
    }
  } catch (...) {
    return set_error(EXPINT_ENOMEM, "host resources exhausted while describing the batched plan");
  }
  if (needed) *needed = text.size() + 1;
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, text.size());
    std::memcpy(buf, text.data(), n);
    buf[n] = 0;
  }
  return EXPINT_OK;
}

extern "C" void expint_batch_plan_destroy(expint_batch_plan* p) {
  if (!p) return;
  free_batch(p);
  delete p;
}
