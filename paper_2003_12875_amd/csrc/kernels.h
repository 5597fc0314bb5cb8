// kernels.h -- what the host runtime sees of the device code: kernel
// argument blocks, launchers and the registry of compiled model shapes.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

#include "plan.h"

namespace nllmi {

// State of a gradient-descent fit (device arrays).
struct GDState {
  double* th_acc;   // n_sets * P  last accepted point
  double* g_acc;    // n_sets * P  its gradient
  double* th_prop;  // n_sets * P  point being evaluated
  double* f_acc;    // n_sets      its NLL (+inf before the first acceptance)
  double* eta;      // n_sets      step size (BHHH: damping lambda)
  int* last_status; // n_sets
  double* b_acc;    // n_sets * P * P  BHHH: matrix at the last accepted point
};

struct SingleArgs {
  const double* cols[kMaxObs];  // SoA event columns (device)
  int64_t n;
  const double* theta;          // n_param (device)
  double* nll_out;              // 1 (device)
  double* grad_out;             // n_param (device) or null
  double* bhhh_out;             // n_param^2 (device): BHHH matrix (evaluation)
  double* partials;             // grid * (NA + 1) double-double pairs
  PerTheta* pt_out;             // per-point constants left by block 0 (evaluation)
  PerTheta* consts;             // fit: constants of the proposal being evaluated,
                                // written by the previous step's finishing kernel
  int* status;                  // accumulated status bits
  const double* glx;            // 256-point Gauss-Legendre rule on [-1, 1]
  const double* glw;
  GDState gd;                   // fit mode: theta = gd.th_prop, set 0
  const double* wsum;           // weighted events: the weights' sum W (device, 1)
  // gradient-descent fit, double-buffered by step parity (k_single_fit):
  const double* partials_prev;  // the previous step's block records (null at the first step)
  GDState gd_out;               // the state the update writes (gd is the one it reads)
  PerTheta* consts_out;         // constants of the proposal this step evaluates
};

// One work item of the batched pass: events [start, end) of one set.
struct WorkItem {
  int64_t start, end;
  int32_t set, flag;  // flag: the offsets were malformed (no events)
};

struct SetsArgs {
  const double* cols[kMaxObs];
  int n_sets;
  const int64_t* offsets;   // n_sets + 1 (device)
  int64_t tile;             // events per work item
  const int64_t* tile_off;  // n_sets + 1 prefix of item counts (device)
  const int* set_flag;      // n_sets: 1 = malformed offsets
  const WorkItem* items;    // tile_off[n_sets] work items in set order
  PerTheta* consts;         // n_sets
  double* partials;         // items * (NA + 1) double-double pairs
  const double* theta;      // n_sets * P (evaluation mode)
  double* nll_out;          // n_sets
  double* grad_out;         // n_sets * P or null
  int* status_out;          // n_sets or null
  GDState gd;               // fit mode
  const double* glx;
  const double* glw;
};

struct VariantOps {
  const char* name;
  int n_leaf, K, nobs, na_grad;
  int kind[kMaxLeaves], obs[kMaxLeaves], root[kMaxLeaves], np[kMaxLeaves];
  int precision;  // 0: FP64 event pass, 1: FP32-compensated
  // lds_cap > 0: LDS reserved per block of the streaming kernel (padded
  // with dynamic LDS), so that at most the intended number of blocks share
  // a CU and the persistent grid spreads evenly over the CUs
  hipError_t (*single)(const Plan&, const SingleArgs&, bool grad, int unroll, int grid, int lds_cap, hipStream_t);
  // fit steps; ev0/ev1 (may be null) are recorded on the stream right before
  // and right after the streaming kernel of the step
  hipError_t (*single_fit)(const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                           hipEvent_t ev0, hipEvent_t ev1);
  hipError_t (*consts)(const Plan&, const double* theta, int n_sets, PerTheta* out, const double* glx,
                       const double* glw, hipStream_t);
  hipError_t (*sets)(const Plan&, const SetsArgs&, bool grad, bool fit, int unroll, int grid, int lds_cap,
                     hipStream_t, hipEvent_t ev0, hipEvent_t ev1);
  hipError_t (*fit_init)(const Plan&, const double* theta, int n_sets, double eta, const GDState&,
                         PerTheta* consts, const double* glx, const double* glw, hipStream_t);
  // BHHH (FP64 shapes with few score features; null where not compiled):
  // NLL, gradient and BHHH matrix at one point, and damped BHHH fit steps
  hipError_t (*single_bhhh)(const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t);
  hipError_t (*single_bhhh_fit)(const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                                hipEvent_t ev0, hipEvent_t ev1);
  int bhhh_record;  // values per block record of the BHHH pass (0: not compiled)
  // weighted events (FP64 shapes; null where not compiled): as single and
  // single_fit, with the weights in SingleArgs::cols[nobs]
  hipError_t (*single_w)(const Plan&, const SingleArgs&, bool grad, int unroll, int grid, int lds_cap, hipStream_t);
  hipError_t (*single_w_fit)(const Plan&, const SingleArgs&, int unroll, int grid, int lds_cap, hipStream_t,
                             hipEvent_t ev0, hipEvent_t ev1);
  // after the last gradient-descent step: the update of the proposal it
  // evaluated (single_fit steps take the previous step's update themselves)
  hipError_t (*fit_finish)(const Plan&, const SingleArgs&, int grid, hipStream_t);
  hipError_t (*w_fit_finish)(const Plan&, const SingleArgs&, int grid, hipStream_t);
};

// registry: every variants_*.hip file appends its compiled shapes
void register_variants_single(std::vector<VariantOps>& out);
void register_variants_mixture(std::vector<VariantOps>& out);
void register_variants_2d(std::vector<VariantOps>& out);
void register_variants_fp32c_1d(std::vector<VariantOps>& out);
void register_variants_fp32c_2d(std::vector<VariantOps>& out);
void register_variants_johnson(std::vector<VariantOps>& out);
void register_variants_chi2(std::vector<VariantOps>& out);

hipError_t launch_schedule(const int64_t* offsets, int n_sets, int64_t n_total, int64_t tile,
                           int64_t* tile_off, int* set_flag, WorkItem* items, hipStream_t st);
hipError_t launch_points(int n_sets, int64_t n, int64_t tile, int64_t* offsets, int64_t* tile_off, int* set_flag,
                         WorkItem* items, hipStream_t st);
hipError_t launch_fit_final(int n_sets, int P, const GDState& gd, double* theta_out, double* nll_out,
                            double* grad_out, int* status_out, hipStream_t st);
// W = sum of n weights into *out (deterministic, compensated): per-block
// partials in part (at most kWsumBlocks double-double pairs), then one block.
constexpr int kWsumBlocks = 1024;
hipError_t launch_wsum(const double* w, int64_t n, double* part, double* out, hipStream_t st);
hipError_t launch_check_range(const double* x, int64_t n, double lo, double hi, unsigned long long* bad,
                              hipStream_t st);

}  // namespace nllmi
