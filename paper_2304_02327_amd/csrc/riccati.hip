// Batched Riccati differential equations, each integrated with ETD2RK phisplit.
//
// Instance i: U' = A1 U + U A2^T + C + U B U with U n1 x n2, B n2 x n1, C n1 x n2
// (paper section 1, eq. Riccati; Kronecker form eq. ODE2d with
// K = I (x) A1 + A2 (x) I, so K u = A1 U + U A2^T and a Tucker operator is
// M1 W M2^T).  One ETD2RK step (section 3.2, eq. ETD2RKtensor read with the
// split factor (2!)^{d-1} = 2 and tau on the whole first bracket) is ten
// GEMM phases; each phase is one persistent grouped launch over all
// instances, longest first:
//    1  T  = U B          (n1 <= n2)   or   B U   (n2 < n1)
//    2  Gn = C + T U                   or   C + U T
//    3  W  = tau A1 U + tau Gn
//    4  W  = W + tau U A2^T
//    5  P  = phi1(tau A1) W
//    6  U2 = U + P phi1(tau A2)^T
//    7  T  = U2 B                      or   B U2
//    8  W2 = tau (T U2 + C - Gn)       or   tau (U2 T + C - Gn)
//    9  P  = phi2(tau A1) W2
//   10  U  = U2 + 2 P phi2(tau A2)^T
// The association of U B U is chosen per instance so the middle product is
// min(n1, n2) square.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.h"

using namespace expint;

namespace {

constexpr int kPhases = 10;
// phases whose B operand is contiguous along k (the others read M^T, contiguous along q)
constexpr bool kPhaseBK[kPhases] = {true, true, true, false, true, false, true, true, true, false};

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
  // descriptors for the current (U, ws)
  void* ddesc = nullptr;      // kPhases * count descriptors
  long* dstart = nullptr;     // kPhases * (count + 1) tile prefix sums
  long phase_tiles[kPhases] = {};
  const void* d_U = nullptr;
  const void* d_ws = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t g_stream = nullptr;
};

namespace {

void free_batch(expint_batch_plan* p) {
  for (double* q : {p->dA1, p->dP1a, p->dP2a, p->dA2, p->dP1b, p->dP2b})
    if (q) (void)hipFree(q);
  if (p->ddesc) (void)hipFree(p->ddesc);
  if (p->dstart) (void)hipFree(p->dstart);
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

// Build the ten phases' descriptors for state U and workspace ws and upload them.
int build_descriptors(expint_batch_plan* p, double* U, char* ws) {
  const size_t dsz = gemm_desc_size();
  const int cnt = p->count;
  std::vector<char> host((size_t)kPhases * cnt * dsz);
  std::vector<long> start((size_t)kPhases * (cnt + 1));
  double* T = reinterpret_cast<double*>(ws);
  double* Gn = T + p->ttotal;
  double* W = Gn + p->total;
  double* P = W + p->total;
  double* U2 = P + p->total;
  double* W2 = U2 + p->total;
  const double tau = p->tau;
  for (int ph = 0; ph < kPhases; ++ph) {
    long acc = 0;
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
      const double *A2 = p->dA2 + p->moff2[i], *P1b = p->dP1b + p->moff2[i], *P2b = p->dP2b + p->moff2[i];
      char* d = host.data() + ((size_t)ph * cnt + slot) * dsz;
      const double* Us = (ph < 6) ? Ui : U2i;  // state the phase reads (phases 7, 8 use U2)
      switch (ph) {
        case 0:
        case 6:  // T = U B  or  B U
          if (left)
            make_gemm_desc(d, Us, n1, Bi, 1, n2, n1, n1, n2, n1, linear(Ti, 1.0));
          else
            make_gemm_desc(d, Bi, n2, Us, 1, n1, n2, n2, n1, n2, linear(Ti, 1.0));
          break;
        case 1:  // Gn = C + T U  or  C + U T
          if (left)
            make_gemm_desc(d, Ti, n1, Ui, 1, n1, n1, n2, n1, n1, linear(Gi, 1.0, Ci, 1.0));
          else
            make_gemm_desc(d, Ui, n1, Ti, 1, n2, n1, n2, n2, n1, linear(Gi, 1.0, Ci, 1.0));
          break;
        case 7:  // W2 = tau (T U2 + C - Gn)  or  tau (U2 T + C - Gn)
          if (left)
            make_gemm_desc(d, Ti, n1, U2i, 1, n1, n1, n2, n1, n1, linear(W2i, tau, Ci, tau, Gi, -tau));
          else
            make_gemm_desc(d, U2i, n1, Ti, 1, n2, n1, n2, n2, n1, linear(W2i, tau, Ci, tau, Gi, -tau));
          break;
        case 2:  // W = tau A1 U + tau Gn
          make_gemm_desc(d, A1, n1, Ui, 1, n1, n1, n2, n1, n1, linear(Wi, tau, Gi, tau));
          break;
        case 3:  // W += tau U A2^T   (B operand A2^T[k, q] = A2[q + n2 k])
          make_gemm_desc(d, Ui, n1, A2, n2, 1, n1, n2, n2, n1, linear(Wi, tau, Wi, 1.0));
          break;
        case 4:  // P = phi1(tau A1) W
          make_gemm_desc(d, P1a, n1, Wi, 1, n1, n1, n2, n1, n1, linear(Pi, 1.0));
          break;
        case 5:  // U2 = U + P phi1(tau A2)^T
          make_gemm_desc(d, Pi, n1, P1b, n2, 1, n1, n2, n2, n1, linear(U2i, 1.0, Ui, 1.0));
          break;
        case 8:  // P = phi2(tau A1) W2
          make_gemm_desc(d, P2a, n1, W2i, 1, n1, n1, n2, n1, n1, linear(Pi, 1.0));
          break;
        case 9:  // U = U2 + 2 P phi2(tau A2)^T
          make_gemm_desc(d, Pi, n1, P2b, n2, 1, n1, n2, n2, n1, linear(Ui, 2.0, U2i, 1.0));
          break;
      }
      start[(size_t)ph * (cnt + 1) + slot] = acc;
      acc += gemm_desc_tiles(d);
    }
    start[(size_t)ph * (cnt + 1) + cnt] = acc;
    p->phase_tiles[ph] = acc;
  }
  // descriptors of an earlier (U, ws) pair may still be read by enqueued work
  if (p->d_U && hipDeviceSynchronize() != hipSuccess)
    return set_error(EXPINT_EHIP, "device synchronisation before a descriptor rebuild failed");
  if (hipMemcpy(p->ddesc, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->dstart, start.data(), start.size() * sizeof(long), hipMemcpyHostToDevice) != hipSuccess)
    return set_error(EXPINT_EHIP, "upload of batched GEMM descriptors failed");
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
  for (int ph = 0; ph < kPhases; ++ph) {
    const char* d = static_cast<const char*>(p->ddesc) + (size_t)ph * p->count * dsz;
    const long* st = p->dstart + (size_t)ph * (p->count + 1);
    const int rc = launch_grouped_gemm(kPhaseBK[ph], d, st, p->count, p->phase_tiles[ph], s);
    if (rc != EXPINT_OK) return rc;
  }
  return EXPINT_OK;
}

int prepare(expint_batch_plan* p, double* U, void* ws) {
  if (!p) return set_error(EXPINT_EINVAL, "plan is NULL");
  if (!U || !ws) return set_error(EXPINT_EINVAL, "U and ws must be non-NULL device pointers");
  if ((reinterpret_cast<uintptr_t>(U) & 15u) || (reinterpret_cast<uintptr_t>(ws) & 15u))
    return set_error(EXPINT_EINVAL, "U and ws must be 16-byte aligned");
  if (p->d_U != U || p->d_ws != ws) return build_descriptors(p, U, static_cast<char*>(ws));
  return EXPINT_OK;
}

}  // namespace

extern "C" int expint_riccati_plan_create(expint_batch_plan** out, int count, const int* n1, const int* n2,
                                          const double* const* A1, const double* const* A2, const double* B,
                                          const double* C, double tau) {
  if (!out) return set_error(EXPINT_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
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
  expint_batch_plan* p = new (std::nothrow) expint_batch_plan();
  if (!p) return set_error(EXPINT_ENOMEM, "plan allocation failed");
  p->count = count;
  p->tau = tau;
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
  auto work = [&](int job) {
    const int i = job / 2;
    const bool first = (job % 2) == 0;
    const int n = first ? n1[i] : n2[i];
    const double* A = first ? A1[i] : A2[i];
    std::vector<double> buf((size_t)3 * n * n);
    phi_setup_single_threaded(true);  // the jobs already run in parallel
    rcs[job] = phi_setup_real(n, A, n, tau, 2, buf.data(), n);
    double* dstA = (first ? hA1.data() + p->moff1[i] : hA2.data() + p->moff2[i]);
    double* dst1 = (first ? hP1a.data() + p->moff1[i] : hP1b.data() + p->moff2[i]);
    double* dst2 = (first ? hP2a.data() + p->moff1[i] : hP2b.data() + p->moff2[i]);
    std::memcpy(dstA, A, sizeof(double) * n * n);
    std::memcpy(dst1, buf.data() + (size_t)n * n, sizeof(double) * n * n);
    std::memcpy(dst2, buf.data() + (size_t)2 * n * n, sizeof(double) * n * n);
  };
  {
    unsigned nt = std::thread::hardware_concurrency();
    nt = nt == 0 ? 1 : (nt > 16 ? 16 : nt);
    std::vector<std::thread> pool;
    std::atomic<int> next{0};
    for (unsigned t = 0; t < nt; ++t)
      pool.emplace_back([&]() {
        for (int job = next++; job < 2 * count; job = next++) work(job);
      });
    for (auto& th : pool) th.join();
  }
  int rc = EXPINT_OK;
  for (int v : rcs)
    if (v != EXPINT_OK) rc = v;
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
  upload(&p->dP1a, hP1a);
  upload(&p->dP2a, hP2a);
  upload(&p->dA2, hA2);
  upload(&p->dP1b, hP1b);
  upload(&p->dP2b, hP2b);
  if (rc == EXPINT_OK && (hipMalloc(&p->ddesc, (size_t)kPhases * count * gemm_desc_size()) != hipSuccess ||
                          hipMalloc(reinterpret_cast<void**>(&p->dstart),
                                    (size_t)kPhases * (count + 1) * sizeof(long)) != hipSuccess))
    rc = set_error(EXPINT_ENOMEM, "device allocation for descriptors failed");
  if (rc != EXPINT_OK) {
    free_batch(p);
    delete p;
    return rc;
  }
  *out = p;
  return EXPINT_OK;
}

extern "C" int expint_batch_state_size(const expint_batch_plan* p, size_t* elements) {
  if (!p || !elements) return set_error(EXPINT_EINVAL, "NULL plan or output");
  *elements = (size_t)p->total;
  return EXPINT_OK;
}

extern "C" int expint_batch_workspace_size(const expint_batch_plan* p, size_t* bytes) {
  if (!p || !bytes) return set_error(EXPINT_EINVAL, "NULL plan or output");
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

extern "C" void expint_batch_plan_destroy(expint_batch_plan* p) {
  if (!p) return;
  free_batch(p);
  delete p;
}
