// runtime.h -- the model object shared by the C ABI (host.cpp) and the
// autotuner (tune.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstring>
#include <vector>

#include "kernels.h"
#include "nll.h"
#include "plan.h"

namespace nllmi {

struct GLTable {
  double* x = nullptr;
  double* w = nullptr;
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void gauss_legendre(int n, double* nodes, double* weights);

}  // namespace nllmi

struct FitKey {
  int mode = 0;  // 1: single-dataset fit, 2: batched fit, 3: single-dataset BHHH fit
  int n_sets = -1;
  const int64_t* offsets = nullptr;
  double* theta = nullptr;
  int n_steps = 0;
  double eta = 0;
  double* nll = nullptr;
  double* grad = nullptr;
  int32_t* status = nullptr;
  nll_schedule sched{};
  int timing = 0;
  bool operator==(const FitKey& o) const {
    return mode == o.mode && n_sets == o.n_sets && offsets == o.offsets && theta == o.theta && n_steps == o.n_steps &&
           eta == o.eta && nll == o.nll && grad == o.grad && status == o.status &&
           timing == o.timing && std::memcmp(&sched, &o.sched, sizeof(sched)) == 0;
  }
};

struct nll_model {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;
  int n_cu = 256;
  int lds_per_cu = 0;       // bytes (0: unknown, no residency cap)
  int lds_per_block = 0;    // largest LDS allocation of one block
  nllmi::Plan plan{};
  const nllmi::VariantOps* ops = nullptr;
  int precision = NLL_FP64;
  nllmi::GLTable gl;

  const double* cols[nllmi::kMaxObs] = {};
  int64_t n = -1;
  const double* weights = nullptr;  // per-event weights (borrowed), or none
  double* wsum = nullptr;           // their sum W (device, 1)
  double* wsum_part = nullptr;      // per-block partials of W (device)
  nll_schedule sched{4, 2, 16384, 16, 2};

  // single dataset
  double* partials = nullptr;       // two halves of partials_half doubles each
  size_t partials_half = 0;
  nllmi::PerTheta* pt_single = nullptr;
  int* status = nullptr;
  unsigned long long* dbad = nullptr;
  int64_t* offsets1 = nullptr;
  int64_t* pts_offsets = nullptr;  // nll_eval_points: virtual offsets s * n
  int pts_cap = 0;

  // many datasets
  int sets_cap = 0;
  int64_t* tile_off = nullptr;
  int* set_flag = nullptr;
  nllmi::WorkItem* items = nullptr;  // batched work items
  size_t items_cap = 0;
  int64_t* chunk_first = nullptr;    // the first item of each chunk of the batched pass
  size_t chunk_cap = 0;
  nllmi::PerTheta* consts = nullptr;
  double* aux = nullptr;  // sets_cap * kAuxWords: a leaf's per-point tables (models with one)
  size_t set_partials_cap = 0;  // bytes
  double* set_partials = nullptr;
  int gd_cap = 0;
  double* gd_mem = nullptr;
  int* gd_status = nullptr;
  double* gd_bacc = nullptr;  // BHHH fits: accepted matrix per set (n_sets * P * P)

  // step timing of fits
  int step_timing = 0;             // 0 off, 1 whole steps, 2 streaming kernels
  std::vector<hipEvent_t> events;  // n_steps + 1 (steps) or 2 n_steps (kernels)
  int timed_steps = -1;
  int timed_mode = 0;

  // recorded fit
  bool use_graph = true;
  bool have_graph = false;
  FitKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};


namespace nllmi {
// Device buffers of one batched pass: the tile schedule (n_sets + 1 prefix
// entries, n_sets flags, the work items), the per-set constants and the
// items' partial records.
struct SetsScratch {
  int64_t* tile_off = nullptr;
  int* set_flag = nullptr;
  WorkItem* items = nullptr;
  int64_t* chunk_first = nullptr;  // chunks + 1
  PerTheta* consts = nullptr;
  double* aux = nullptr;  // n_sets * kAuxWords (models with per-point tables)
  double* partials = nullptr;
};
// argument checks of the batched evaluation (no device work)
nll_status batched_args_ok(const nll_model* m, int32_t n_sets, const int64_t* offsets, const double* theta,
                           const double* nll_out);
// most work items n_sets consecutive event ranges of the attached data can need
int64_t batched_items_bound(const nll_model* m, int32_t n_sets);
// bytes of one item's partial record
size_t batched_record_bytes(const nll_model* m);
// enqueue the batched pass on the model's stream with the given buffers
// (nothing is allocated)
nll_status eval_batched_on(nll_model* m, int32_t n_sets, const int64_t* offsets, const double* theta,
                           double* nll_out, double* grad_out, int32_t* status_out, const SetsScratch& s);
nll_status tune_model(nll_model* m, int which, int n_sets, const int64_t* offsets, const double* theta);
}  // namespace nllmi
