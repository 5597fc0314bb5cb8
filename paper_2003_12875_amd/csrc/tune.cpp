// tune.cpp -- launch-schedule autotuner.
//
// Candidates: single dataset -- events per thread per tile (2, 4, 8) x
// blocks per CU (1..16); batched -- events per thread per tile x events per
// chunk (8k..32k) x blocks per CU.  Each candidate is first checked
// against the default schedule's result (only the summation order differs:
// relative NLL difference <= 1e-12 per dataset in FP64; in the
// FP32-compensated mode, where the order also regroups the single-precision
// per-thread sums, within that mode's accuracy, max(1e-9, 1e-6/sqrt(N)) for
// one dataset and 1e-6 for sets) and then timed with HIP events over several
// evaluations; the fastest passing candidate is kept.  Choices are cached in a plain text
// file named by $NLLMI_TUNE_CACHE, one line per (shape, precision, mode,
// log2 event count) key.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "nll.h"
#include "runtime.h"

namespace nllmi {
namespace {

std::string cache_key(const nll_model* m, int which) {
  int bucket = 0;
  for (int64_t n = m->n; n > 1; n >>= 1) ++bucket;
  std::ostringstream os;
  os << "s5|" << m->ops->name << "|p" << m->precision << "|w" << which << "|b" << bucket;  // s5: 5-field schedule
  std::string k = os.str();
  for (char& c : k)
    if (c == ' ') c = '_';
  return k;
}

bool cache_lookup(const std::string& key, nll_schedule* out) {
  const char* path = std::getenv("NLLMI_TUNE_CACHE");
  if (!path || std::getenv("NLLMI_TUNE_FORCE")) return false;
  std::ifstream f(path);
  std::string k;
  nll_schedule s{};
  while (f >> k >> s.unroll >> s.blocks_per_cu >> s.tile_events >> s.sets_blocks_per_cu >> s.sets_unroll)
    if (k == key) {
      *out = s;
      return true;
    }
  return false;
}

void cache_store(const std::string& key, const nll_schedule& s) {
  const char* path = std::getenv("NLLMI_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << s.unroll << ' ' << s.blocks_per_cu << ' ' << s.tile_events << ' ' << s.sets_blocks_per_cu
    << ' ' << s.sets_unroll
    << '\n';
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

bool close_rel(double x, double y, double tol) {
  if (!std::isfinite(x) || !std::isfinite(y)) return x == y;
  return std::fabs(x - y) <= tol * std::fmax(1.0, std::fabs(y));
}

}  // namespace

nll_status tune_model(nll_model* m, int which, int n_sets, const int64_t* offsets, const double* theta) {
  const std::string key = cache_key(m, which);
  nll_schedule cached;
  if (cache_lookup(key, &cached)) return nll_set_schedule(m, &cached);
  if (!theta) return NLL_ERR_ARG;
  if (which == 2 && (n_sets < 1 || !offsets)) return NLL_ERR_ARG;
  const int P = m->plan.n_param;
  const int S = which == 1 ? 1 : n_sets;
  double *d_nll = nullptr, *d_grad = nullptr;
  if (hipMalloc(&d_nll, sizeof(double) * S) != hipSuccess) return NLL_ERR_OOM;
  if (hipMalloc(&d_grad, sizeof(double) * S * P) != hipSuccess) {
    (void)hipFree(d_nll);
    return NLL_ERR_OOM;
  }
  auto run = [&]() -> nll_status {
    if (which == 1) return nll_eval_grad(m, theta, d_nll, d_grad);
    return nll_eval_batched(m, n_sets, offsets, theta, d_nll, d_grad, nullptr);
  };
  std::vector<double> ref(S), got(S);
  double tol = 1e-12;
  if (m->precision == NLL_FP32C)
    tol = which == 1 ? std::fmax(1e-9, 1e-6 / std::sqrt((double)std::max<int64_t>(m->n, 1))) : 1e-6;
  const nll_schedule base = m->sched;
  nll_schedule best = base;
  float best_ms = 1e30f;
  nll_status st = run();
  if (st == NLL_OK && hipStreamSynchronize(m->stream) == hipSuccess &&
      hipMemcpy(ref.data(), d_nll, sizeof(double) * S, hipMemcpyDeviceToHost) == hipSuccess) {
    std::vector<nll_schedule> cands;
    if (which == 1) {
      for (int u : {2, 4, 8})
        for (int b : {1, 2, 3, 4, 8, 16})
          cands.push_back(nll_schedule{u, b, base.tile_events, base.sets_blocks_per_cu, base.sets_unroll});
    } else {
      for (int u : {2, 4, 8})
        for (int t : {8192, 16384, 32768})
          for (int b : {2, 3, 4, 8})
            cands.push_back(nll_schedule{base.unroll, base.blocks_per_cu, t, b, u});
    }
    Timer tm;
    for (const nll_schedule& c : cands) {
      if (nll_set_schedule(m, &c) != NLL_OK) continue;
      if (run() != NLL_OK || hipStreamSynchronize(m->stream) != hipSuccess) continue;
      if (hipMemcpy(got.data(), d_nll, sizeof(double) * S, hipMemcpyDeviceToHost) != hipSuccess) continue;
      bool ok = true;
      for (int s = 0; s < S && ok; ++s) ok = close_rel(got[s], ref[s], tol);
      if (!ok) continue;  // a schedule must reproduce the reference first
      const int reps = which == 1 ? 20 : 5;
      (void)hipEventRecord(tm.a, m->stream);
      for (int r = 0; r < reps; ++r) run();
      (void)hipEventRecord(tm.b, m->stream);
      (void)hipEventSynchronize(tm.b);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, tm.a, tm.b);
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  }
  (void)hipFree(d_nll);
  (void)hipFree(d_grad);
  nll_set_schedule(m, &best);
  if (best_ms < 1e30f) cache_store(key, best);
  return st;
}

}  // namespace nllmi
