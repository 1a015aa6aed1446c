// The autotuner: picks the launch configuration (tile shape, waves, pipeline
// depth, whether modes 1 and 2 share a launch) of each kernel family per launch
// shape by timing every candidate on the device, and keeps the choice for the
// life of the process (and, with EXPINT_TUNE_CACHE=path, across processes).
//
// Every candidate of a family computes the same sums in the same order (the
// K loop runs in index order whatever the tile; the int8 level sums are exact),
// so a tuned choice changes the time of a launch, never its result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace expint {
namespace {

// Scratch operands for timing: uniform values in [-1/2, 1/2) from a hash of the
// index (MFMA power, and so the clock the chip holds, depends on the data; zeros
// would time optimistically).
__global__ void k_fill_hash(double* __restrict__ x, long n, unsigned seed) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    unsigned h = (unsigned)i * 0x9E3779B1u ^ seed;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    h *= 0xC2B2AE3Du;
    h ^= h >> 16;
    x[i] = (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
  }
}

struct Entry {
  int choice;
  double us;
};
using FullKey = std::tuple<std::string, int, long, long, long, long>;

std::mutex g_table_mutex;
std::map<FullKey, Entry> g_table;
bool g_cache_loaded = false;
std::mutex g_tune_mutex;  // one tuning run at a time (timings must not overlap)

thread_local int t_forced_family = -1;
thread_local int t_forced_choice = -1;

const char* const kFamilyTags[TUNE_FAMILIES] = {"mp_real", "mp_cplx",   "sliced", "modes12",
                                                "lp_fp32", "lp_bf16x3", "grouped"};
const char* const kFamilyEnv[TUNE_FAMILIES] = {"EXPINT_TILE",    "EXPINT_TILE",    "EXPINT_SLICE_TILE", "EXPINT_M12",
                                               "EXPINT_LP_TILE", "EXPINT_LP_TILE", "EXPINT_GROUPED"};

// gcnArchName of the current device (cached per device ordinal)
std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lock(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    name = prop.gcnArchName;
    const size_t colon = name.find(':');
    if (colon != std::string::npos) name.resize(colon);
  }
  names[dev] = name;
  return name;
}

FullKey full_key(const TuneKey& k) { return FullKey(device_arch(), k.family, k.a, k.b, k.c, k.d); }

int candidate_index(int family, const char* name) {
  for (int i = 0; i < tune_candidate_count(family); ++i)
    if (std::strcmp(name, tune_candidate_name(family, i)) == 0) return i;
  return -1;
}

// EXPINT_TUNE_CACHE: one line per entry, "arch family a b c d candidate us"
void load_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = std::getenv("EXPINT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64], fam[32], cand[64];
  long a, b, c, d;
  double us;
  while (std::fscanf(f, "%63s %31s %ld %ld %ld %ld %63s %lf", arch, fam, &a, &b, &c, &d, cand, &us) == 8) {
    int family = -1;
    for (int i = 0; i < TUNE_FAMILIES; ++i)
      if (std::strcmp(fam, kFamilyTags[i]) == 0) family = i;
    if (family < 0) continue;
    const int choice = candidate_index(family, cand);
    if (choice < 0) continue;
    g_table.emplace(FullKey(arch, family, a, b, c, d), Entry{choice, us});  // the first line of a key wins
  }
  std::fclose(f);
}

void append_cache(const FullKey& fk, const Entry& e) {
  const char* path = std::getenv("EXPINT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %s %ld %ld %ld %ld %s %.3f\n", std::get<0>(fk).c_str(), kFamilyTags[std::get<1>(fk)],
               std::get<2>(fk), std::get<3>(fk), std::get<4>(fk), std::get<5>(fk),
               tune_candidate_name(std::get<1>(fk), e.choice), e.us);
  std::fclose(f);
}

}  // namespace

int tune_candidate_count(int family) {
  switch (family) {
    case TUNE_MP_REAL:
    case TUNE_MP_CPLX: return mode_product_tile_count();
    case TUNE_SLICED: return sliced_tile_count();
    case TUNE_MODES12: return modes12_shape_count() + 1;
    case TUNE_LP_FP32: return lp_tile_count(EXPINT_PREC_FP32);
    case TUNE_LP_BF16X3: return lp_tile_count(EXPINT_PREC_BF16X3);
    case TUNE_GROUPED: return grouped_scheme_count();
    default: return 0;
  }
}

const char* tune_candidate_name(int family, int i) {
  switch (family) {
    case TUNE_MP_REAL:
    case TUNE_MP_CPLX: return mode_product_tile_name(i);
    case TUNE_SLICED: return sliced_tile_name(i);
    case TUNE_MODES12: return i == modes12_shape_count() ? "off" : modes12_shape_name(i);
    case TUNE_LP_FP32: return lp_tile_name(EXPINT_PREC_FP32, i);
    case TUNE_LP_BF16X3: return lp_tile_name(EXPINT_PREC_BF16X3, i);
    case TUNE_GROUPED: return grouped_scheme_name(i);
    default: return "?";
  }
}

int tune_lookup(const TuneKey& k) {
  const FullKey fk = full_key(k);
  std::lock_guard<std::mutex> lock(g_table_mutex);
  load_cache_locked();
  auto it = g_table.find(fk);
  return it == g_table.end() ? -1 : it->second.choice;
}

int tune_choice(const TuneKey& k) {
  if (t_forced_family == k.family && t_forced_choice >= 0) return t_forced_choice;
  if (const char* e = std::getenv(kFamilyEnv[k.family])) {
    const int i = candidate_index(k.family, e);
    if (i >= 0) return i;
  }
  return tune_lookup(k);
}

namespace {

// Average microseconds of one call of `launch` on stream st (HIP events),
// after one untimed call; enough calls for about 2 ms of work (2 .. 20).
int time_launch(hipStream_t st, const std::function<int()>& launch, double* us) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = EXPINT_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = set_error(EXPINT_EHIP, "tuning: event creation failed");
  }
  float ms = 0.f;
  int reps = 1;
  if (rc == EXPINT_OK) rc = launch();
  if (rc == EXPINT_OK && (hipEventRecord(e0, st) != hipSuccess || (rc = launch()) != EXPINT_OK ||
                          hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = rc != EXPINT_OK ? rc : set_error(EXPINT_EHIP, "tuning: timing failed");
  if (rc == EXPINT_OK) {
    reps = std::min(20, std::max(2, (int)(2.0 / std::max(ms, 1e-3f))));
    if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(EXPINT_EHIP, "tuning: timing failed");
    for (int i = 0; i < reps && rc == EXPINT_OK; ++i) rc = launch();
    if (rc == EXPINT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = set_error(EXPINT_EHIP, "tuning: timing failed");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == EXPINT_OK) *us = 1e3 * ms / reps;
  return rc;
}

}  // namespace

// Times every candidate of k's family for the launches `launch` makes (each
// call: one launch configuration of that family, as tune_choice forces it) and
// keeps the fastest (the lower index on a tie).  A key tuned before (in this
// process or the cache file) is not timed again.
int tune_key(const TuneKey& k, void* stream, const std::function<int()>& launch) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (tune_lookup(k) >= 0) return EXPINT_OK;
  const int nc = tune_candidate_count(k.family);
  int best = -1;
  double best_us = 0.0;
  int rc = EXPINT_OK;
  for (int i = 0; i < nc && rc == EXPINT_OK; ++i) {
    t_forced_family = k.family;
    t_forced_choice = i;
    double us = 0.0;
    rc = time_launch(st, launch, &us);
    if (rc == EXPINT_OK && (best < 0 || us < best_us)) {
      best = i;
      best_us = us;
    }
  }
  t_forced_family = -1;
  t_forced_choice = -1;
  if (rc != EXPINT_OK) return rc;
  const FullKey fk = full_key(k);
  // kept at the cache file's precision, so that this process and one that reads the file agree
  const Entry e{best, std::round(best_us * 1e3) / 1e3};
  bool added = false;
  {
    std::lock_guard<std::mutex> lock(g_table_mutex);
    load_cache_locked();
    added = g_table.emplace(fk, e).second;
  }
  if (added) append_cache(fk, e);
  return EXPINT_OK;
}

// Tunes every launch a Tucker operator (every mode present) of this shape,
// element type and precision makes, on scratch tensors and matrices of the
// same sizes filled with hashed values.
// Synchronous; allocates and frees its scratch.
int tune_tucker_shapes(int d, const int* n, int dtype, int precision, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool cplx = dtype == EXPINT_C128;
  const bool lp = precision == EXPINT_PREC_FP32 || precision == EXPINT_PREC_BF16X3;
  if (lp && cplx) return EXPINT_OK;  // complex64 products have one configuration
  std::lock_guard<std::mutex> serial(g_tune_mutex);
  const size_t es = cplx ? 16 : 8;
  long N = 1;
  int nmax = 1;
  for (int mu = 0; mu < d; ++mu) {
    N *= n[mu];
    nmax = std::max(nmax, n[mu]);
  }
  std::vector<void*> owned;
  unsigned seed = 1;
  auto alloc = [&](size_t bytes, void** p) {
    *p = nullptr;
    bytes = std::max<size_t>(bytes, 256);
    if (hipMalloc(p, bytes) != hipSuccess) return set_error(EXPINT_ENOMEM, "tuning: device allocation failed");
    owned.push_back(*p);
    const long count = (long)(bytes / 8);
    const long blocks = std::min<long>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_hash, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<double*>(*p), count, seed++);
    if (hipGetLastError() != hipSuccess) return set_error(EXPINT_EHIP, "tuning: scratch fill failed");
    return EXPINT_OK;
  };
  void *X, *Y, *Z, *Mm;
  int rc = alloc((size_t)N * es, &X);
  if (rc == EXPINT_OK) rc = alloc((size_t)N * es, &Y);
  if (rc == EXPINT_OK) rc = alloc((size_t)N * es, &Z);
  if (rc == EXPINT_OK) rc = alloc((size_t)nmax * nmax * es, &Mm);
  void *dig = nullptr, *mdig = nullptr;
  if (rc == EXPINT_OK && precision == EXPINT_PREC_SLICED) {
    size_t b = 0;
    for (int mu = 0; mu < d; ++mu) b = std::max(b, slice_digits_bytes(N / n[mu], n[mu]));
    rc = alloc(b, &dig);
    if (rc == EXPINT_OK) rc = alloc(slice_digits_bytes(nmax, nmax), &mdig);
  }
  Epilogue plain;
  plain.op = EPI_AXPBY;
  plain.alpha = 1.0;
  plain.beta = 0.0;
  plain.out0 = Y;
  for (int mu = 0; mu < d && rc == EXPINT_OK; ++mu) {
    long s = 1, r = 1;
    for (int k = 0; k < mu; ++k) s *= n[k];
    for (int k = mu + 1; k < d; ++k) r *= n[k];
    if (lp) {
      // as in a chain: the first mode reads FP64, the inner ones FP32, the last one
      // returns FP64 (timed with a plain store)
      const bool v32 = mu > 0, out32 = mu + 1 < d;
      rc = tune_key(lp_key(precision, s, n[mu], r), st, [&]() {
        return launch_mode_product_lp(precision, false, v32, out32, s, n[mu], r, Mm, X, plain, st);
      });
    } else if (precision == EXPINT_PREC_SLICED) {
      rc = launch_slice(static_cast<const double*>(Mm), n[mu], n[mu], 1, false, mdig, st);
      if (rc == EXPINT_OK) rc = launch_slice(static_cast<const double*>(X), s, n[mu], r, mu == 0, dig, st);
      if (rc == EXPINT_OK)
        rc = tune_key(sliced_key(s, n[mu], r), st,
                      [&]() { return launch_sliced_mode_product(s, n[mu], r, mu == 0, mdig, dig, plain, st); });
    } else {
      rc = tune_key(mode_product_key(cplx, s, n[mu], r), st,
                    [&]() { return launch_mode_product(dtype, s, n[mu], r, Mm, X, plain, st); });
    }
  }
  if (rc == EXPINT_OK && precision == EXPINT_PREC_FP64 && !cplx && d >= 2 && modes12_fits(n[0], n[1])) {
    long r = 1;
    for (int k = 2; k < d; ++k) r *= n[k];
    const int off = modes12_shape_count();
    rc = tune_key(modes12_key(n[0], n[1], r), st, [&]() {
      if (tune_choice(modes12_key(n[0], n[1], r)) == off) {  // two single-mode launches
        Epilogue e1 = plain;
        e1.out0 = Z;
        const int r1 = launch_mode_product(dtype, 1, n[0], N / n[0], Mm, X, e1, st);
        return r1 != EXPINT_OK ? r1 : launch_mode_product(dtype, n[0], n[1], r, Mm, Z, plain, st);
      }
      return launch_modes12(n[0], n[1], r, Mm, Mm, X, plain, st);
    });
  }
  if (hipStreamSynchronize(st) != hipSuccess && rc == EXPINT_OK) rc = set_error(EXPINT_EHIP, "tuning: synchronisation failed");
  for (void* p : owned) (void)hipFree(p);
  return rc;
}

// One line per tuned key of the current device's architecture and of the shape's
// families, "family a b c d -> candidate (us)"; used by expint_plan_describe.
std::string tune_describe(const TuneKey& k) {
  const FullKey fk = full_key(k);
  std::lock_guard<std::mutex> lock(g_table_mutex);
  load_cache_locked();
  char buf[192];
  auto it = g_table.find(fk);
  if (it == g_table.end()) {
    std::snprintf(buf, sizeof(buf), "%s %ld %ld %ld %ld: default", kFamilyTags[k.family], k.a, k.b, k.c, k.d);
  } else {
    std::snprintf(buf, sizeof(buf), "%s %ld %ld %ld %ld: %s (tuned, %.1f us)", kFamilyTags[k.family], k.a, k.b,
                  k.c, k.d, tune_candidate_name(k.family, it->second.choice), it->second.us);
  }
  return buf;
}

}  // namespace expint

using namespace expint;

extern "C" int tucker_tune(int d, const int* n, int dtype, int precision, void* stream) {
  if (d < 1 || d > 4 || !n) return set_error(EXPINT_EINVAL, "tucker_tune: need 1 <= d <= 4 and a size array");
  long N = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1) return set_error(EXPINT_EINVAL, "tucker_tune: n[%d] = %d must be >= 1", mu, n[mu]);
    N *= n[mu];
    if (N >= (1L << 31)) return set_error(EXPINT_EINVAL, "tucker_tune: tensor too large");
  }
  if (dtype != EXPINT_F64 && dtype != EXPINT_C128) return set_error(EXPINT_EINVAL, "tucker_tune: unknown dtype %d", dtype);
  if (precision < EXPINT_PREC_FP64 || precision > EXPINT_PREC_SLICED)
    return set_error(EXPINT_EINVAL, "tucker_tune: unknown precision %d", precision);
  if (precision == EXPINT_PREC_SLICED && dtype != EXPINT_F64)
    return set_error(EXPINT_ENOTSUP, "tucker_tune: exact slice is for real data");
  if ((size_t)N * (dtype == EXPINT_C128 ? 16 : 8) >= (1ull << 31))
    return set_error(EXPINT_ENOTSUP, "tucker_tune: a tensor above 2 GiB exceeds the operand limit");
  if (precision == EXPINT_PREC_SLICED)
    for (int mu = 0; mu < d; ++mu)
      if (n[mu] > kSliceMaxK) return set_error(EXPINT_ENOTSUP, "tucker_tune: n[%d] exceeds %d", mu, kSliceMaxK);
  return tune_tucker_shapes(d, n, dtype, precision, stream);
}
