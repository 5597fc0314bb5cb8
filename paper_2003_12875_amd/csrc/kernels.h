// kernels.h -- what the host runtime sees of the device code: kernel
// argument blocks, launchers and the registry of compiled model shapes.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

#include "args.h"
#include "plan.h"

namespace nllmi {

struct VariantOps {
  const char* name;
  int n_leaf, K, nobs, na_grad;
  int kind[kMaxLeaves], obs[kMaxLeaves], root[kMaxLeaves], np[kMaxLeaves];
  int precision;  // 0: FP64 event pass, 1: FP32-compensated
  // 1: term k is the k-th non-root leaf (with the root factors), as the
  // kernels then assume; 0: the plan's term masks define the terms
  int flat;
  // 1: a leaf keeps per-point tables (kAuxWords) beside PerTheta, passed
  // as SingleArgs::aux / SetsArgs::aux and to consts / fit_init
  int aux;
  // threads per block of the per-set finishing kernel (finish_threads<M>)
  int fin_threads;
  // run-time compiled shapes: their module and kernels (null: compiled
  // ahead of time); the launchers receive the variant itself
  const void* rtc;
  // lds_cap > 0: LDS reserved per block of the streaming kernel (padded
  // with dynamic LDS), so that at most the intended number of blocks share
  // a CU and the persistent grid spreads evenly over the CUs
  hipError_t (*single)(const VariantOps&, const Plan&, const SingleArgs&, bool grad, int unroll, int grid, int lds_cap, hipStream_t);
  // fit steps; ev0/ev1 (may be null) are recorded on the stream right before
  // and right after the streaming kernel of the step
  hipError_t (*single_fit)(const VariantOps&, const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                           hipEvent_t ev0, hipEvent_t ev1);
  hipError_t (*consts)(const VariantOps&, const Plan&, const double* theta, int n_sets, PerTheta* out, double* aux,
                       const double* glx, const double* glw, hipStream_t);
  hipError_t (*sets)(const VariantOps&, const Plan&, const SetsArgs&, bool grad, bool fit, int unroll, int grid, int lds_cap,
                     hipStream_t, hipEvent_t ev0, hipEvent_t ev1);
  hipError_t (*fit_init)(const VariantOps&, const Plan&, const double* theta, int n_sets, double eta, const GDState&,
                         PerTheta* consts, double* aux, const double* glx, const double* glw, hipStream_t);
  // BHHH (FP64 shapes with few score features; null where not compiled):
  // NLL, gradient and BHHH matrix at one point, and damped BHHH fit steps
  hipError_t (*single_bhhh)(const VariantOps&, const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t);
  hipError_t (*single_bhhh_fit)(const VariantOps&, const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                                hipEvent_t ev0, hipEvent_t ev1);
  int bhhh_record;  // values per block record of the BHHH pass (0: not compiled)
  // weighted events (FP64 shapes; null where not compiled): as single and
  // single_fit, with the weights in SingleArgs::cols[nobs]
  hipError_t (*single_w)(const VariantOps&, const Plan&, const SingleArgs&, bool grad, int unroll, int grid, int lds_cap, hipStream_t);
  hipError_t (*single_w_fit)(const VariantOps&, const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                             hipEvent_t ev0, hipEvent_t ev1);
  // after the last gradient-descent step: the update of the proposal it
  // evaluated (single_fit steps take the previous step's update themselves)
  hipError_t (*fit_finish)(const VariantOps&, const Plan&, const SingleArgs&, int grid, hipStream_t);
  hipError_t (*w_fit_finish)(const VariantOps&, const Plan&, const SingleArgs&, int grid, hipStream_t);
};

// registry: every variants_*.hip file appends its compiled shapes
void register_variants_single(std::vector<VariantOps>& out);
void register_variants_mixture(std::vector<VariantOps>& out);
void register_variants_2d(std::vector<VariantOps>& out);
void register_variants_fp32c_1d(std::vector<VariantOps>& out);
void register_variants_fp32c_2d(std::vector<VariantOps>& out);
void register_variants_johnson(std::vector<VariantOps>& out);
void register_variants_chi2(std::vector<VariantOps>& out);
void register_variants_hypatia(std::vector<VariantOps>& out);

// work items of the batched pass over the chunks of g (see common.hip),
// chunk_first[G K + 1]
hipError_t launch_schedule(const int64_t* offsets, int n_sets, const ChunkGrid& g, int64_t* tile_off,
                           int* set_flag, WorkItem* items, int64_t* chunk_first, hipStream_t st);
// points mode: one round of G chunks (chunk_first[G + 1])
hipError_t launch_points(int n_sets, int64_t n, int64_t tile, int G, int64_t* offsets, int64_t* tile_off,
                         int* set_flag, WorkItem* items, int64_t* chunk_first, hipStream_t st);
hipError_t launch_fit_final(int n_sets, int P, const GDState& gd, double* theta_out, double* nll_out,
                            double* grad_out, int* status_out, hipStream_t st);
// W = sum of n weights into *out (deterministic, compensated): per-block
// partials in part (at most kWsumBlocks double-double pairs), then one block.
constexpr int kWsumBlocks = 1024;
hipError_t launch_wsum(const double* w, int64_t n, double* part, double* out, hipStream_t st);
// read-bandwidth probe: n doubles (16-byte aligned) once, one sum per block into out[blocks]
hipError_t launch_read_probe(const double* x, int64_t n, double* out, int blocks, hipStream_t st);
hipError_t launch_check_range(const double* x, int64_t n, double lo, double hi, unsigned long long* bad,
                              hipStream_t st);

}  // namespace nllmi
