// histfactory.h -- plain data of the binned template likelihood (the
// HistFactory-type binned models the paper names as the next target of its
// work, Summary; built from histograms, Sec. 1), shared by the host runtime
// and the device kernels.
//
//   nu_b = sum_s F_s(theta) T_sb + sum_h c_h(theta) d_hb
//   NLL  = sum_b (nu_b - n_b ln nu_b) + 1/2 sum_{constrained p} (theta_p - m_p)^2 / s_p^2
// and, with per-bin statistical parameters (HistFactory's staterror), the
// flagged samples' terms of bin b times gamma_b, plus
// 1/2 sum_b (gamma_b - 1)^2 / sigma_b^2 over the bins that have one (or,
// HistFactory's shapesys, sum_b tau_b (gamma_b - ln gamma_b), tau = 1/sigma^2).
//
// F_s: the sample's normfactors times its normsys factors
// (eta = hi^alpha for alpha >= 0, lo^-alpha below); histosys h on sample
// s_h with parameter alpha_h adds alpha_h (up - T) or alpha_h (T - down)
// to the sample's bins, i.e. c_h = F_{s_h} alpha_h times the delta template
// d_hb of alpha_h's side.  The streaming pass accumulates, besides the
// NLL, the per-sample sums ST_s = sum_b w_b T_sb and per-histosys sums
// SD_h = sum_b w_b d_hb with w_b = 1 - n_b/nu_b; every parameter
// derivative is assembled from them after the reduction.
//
// Smooth codes: a normsys factor is, for |alpha| < 1, a sixth-order
// polynomial meeting hi^alpha and lo^-alpha at +-1 with equal value, slope
// and curvature; a histosys delta is c_u du + c_d dd with both templates
// (du = up - T, dd = T - down) weighted by polynomials of alpha for
// |alpha| < 1 (linear beyond).  A model with a smooth histosys sums both
// templates apart per histosys (U_h, L_h in the record's histosys slots, at
// most kHfPolyHisto of them), so that value and derivative coefficients
// can both be applied after the reduction.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "plan.h"

namespace nllmi {

constexpr int kHfMaxSamples = 8;
constexpr int kHfMaxHisto = 24;
constexpr int kHfPolyHisto = kHfMaxHisto / 2;  // histosys of a model with the smooth code
constexpr int kHfMaxNormsys = 16;
constexpr int kHfMaxNormfactor = 8;
// block record: NLL, ST_s, SD_h (smooth: U_h, L_h pairs), invalid-bin count
constexpr int kHfNV = 1 + kHfMaxSamples + kHfMaxHisto + 1;

// Modifiers are sorted by sample on the host, so that sample s owns the
// index ranges [x_start[s], x_start[s + 1]) of each kind; each parameter's
// modifiers are listed as contribution slots (normfactors 0.., normsys
// kHfMaxNormfactor.., histosys kHfMaxNormfactor + kHfMaxNormsys..).
constexpr int kHfSlots = kHfMaxNormfactor + kHfMaxNormsys + kHfMaxHisto;
struct HFPlan {
  int32_t n_samples, n_histo, n_normsys, n_normfactor, n_param;
  int32_t nf_start[kHfMaxSamples + 1], ns_start[kHfMaxSamples + 1], hs_start[kHfMaxSamples + 1];
  int32_t nf_sample[kHfMaxNormfactor], nf_param[kHfMaxNormfactor];
  int32_t ns_sample[kHfMaxNormsys], ns_param[kHfMaxNormsys];
  int32_t histo_sample[kHfMaxHisto], histo_param[kHfMaxHisto];
  int32_t par_start[kMaxParams + 1], par_slot[kHfSlots];
  int32_t par_free[kMaxParams], par_constrained[kMaxParams];
  int32_t stat_mask;  // samples scaled by the per-bin statistical parameters gamma_b
  int32_t stat_kind;  // their constraint: 0 Gaussian (staterror), 1 Poisson (shapesys)
  int32_t ns_code[kHfMaxNormsys], hs_code[kHfMaxHisto];  // 0: hi^a / lo^-a, linear; 1: smooth
  int32_t smooth_histo;  // 1: some histosys uses the smooth code (both templates summed apart)
  double ns_lnhi[kHfMaxNormsys], ns_lnlo[kHfMaxNormsys];
  double par_lo[kMaxParams], par_hi[kMaxParams];
  double par_mean[kMaxParams], par_ivar[kMaxParams];  // constraint mean and 1 / width^2
};

struct HFArgs {
  int64_t n_bins;
  const double* counts;                 // n_b (caller's)
  const double* nominal[kHfMaxSamples]; // T_sb (caller's)
  const double* dup[kHfMaxHisto];       // up - T (library's), in sorted order
  const double* ddn[kHfMaxHisto];       // T - down (library's)
  const double* theta;                  // n_param
  double* nll_out;
  double* grad_out;                     // n_param or null
  double* partials;                     // grid * kHfNV double-double pairs
  int* status;                          // accumulated status bits
  // per-bin statistical parameters (nll_hf_eval_stat): gamma_b (caller's),
  // tau_b = 1/sigma_b^2 (library's; < 0 where the bin has none), and
  // d NLL / d gamma_b (caller's, n_bins, or null)
  const double* gamma;
  const double* stat_tau;
  double* grad_gamma;
};

hipError_t launch_hf_deltas(const double* nominal, const double* up, const double* down, int64_t n, double* dup,
                            double* ddn, hipStream_t st);
hipError_t launch_hf_eval(const HFPlan& pl, const HFArgs& a, bool grad, int grid, hipStream_t st);
hipError_t launch_hf_tau(const double* sigma, int64_t n, double* tau, hipStream_t st);

}  // namespace nllmi
