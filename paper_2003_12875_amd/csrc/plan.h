// plan.h -- plain data shared by the host runtime and the device kernels.
//
// A model graph (observables, parameters, leaf densities, sums, products;
// the computation graph of the paper's Sec. 1) is lowered on the host into
// a "sum of products" plan:
//
//     p(x) = sum_k  w_k(theta)  prod_{l in S_k}  g_l(x) / Z_l(theta)
//
// where every leaf l is one of the built-in densities, w_k is a product of
// sum coefficients along the path to term k, and Z_l is the normalisation
// integral of leaf l over its observable range.  Leaves present in every
// term ("root factors") are kept out of the per-event log-sum-exp.
//
// Per parameter point the device computes a PerTheta block of constants
// once (the node-local caching of parameter-only branches described in
// Sec. 5.1); the per-event pass only reads it.
#pragma once

#include <stdint.h>

namespace nllmi {

constexpr int kMaxObs = 4;
constexpr int kMaxParams = 32;
constexpr int kMaxLeaves = 8;
constexpr int kMaxTerms = 8;
constexpr int kMaxLeafParams = 12;
constexpr int kLeafConsts = 12;     // per-event constants of one leaf
constexpr int kMaxSums = 4;
constexpr int kMaxSumChildren = 8;
constexpr int kMaxPathRefs = 4;     // sum coefficients on the path to a term
constexpr int kBlock = 256;         // threads per block (4 wave64)
constexpr int kFinishBlock = 1024;  // threads of the single-dataset finishing kernel
constexpr int kMaxAcc = 1 + kMaxTerms + kMaxLeaves * kMaxLeafParams;

enum LeafKind : int32_t {
  kGauss = 1, kExp = 2, kCheb = 3, kCB = 4, kArgus = 5, kJohnson = 8, kChi2 = 9, kHypatia = 10, kJit = 11
};
constexpr int kJitMaxLeafParams = 8;  // parameters of a formula leaf (forward-mode duals)
constexpr int kJitMaxPanels = 256;    // panels of its composite Gauss-Legendre normalisation

// Hypatia2 per-point tables (at most one such leaf per model; kept beside
// PerTheta, in LDS or in a per-set device array): Chebyshev interpolants of
// three functions of log z on up to kHypPanels panels of degree
// kHypDeg - 1, then scalars and the tails' derivative tables
constexpr int kHypDeg = 16;
constexpr int kHypPanels = 8;
constexpr int kHypCoef = 3 * kHypPanels * kHypDeg;
constexpr int kHypScal = kHypCoef;          // 32 scalars
constexpr int kHypTails = kHypCoef + 32;    // 2 x 9 x 3 tail coefficients
constexpr int kAuxWords = kHypCoef + 32 + 54 + 2;
enum NormKind : int32_t { kNormAnalytic = 0, kNormGL = 1, kNormGLSingle = 2 };

// Runtime description of one lowered model (kernel argument, by value).
struct Plan {
  int32_t n_obs;
  double lo[kMaxObs], hi[kMaxObs];
  int32_t n_param;
  double par_lo[kMaxParams], par_hi[kMaxParams];
  int32_t par_free[kMaxParams];

  int32_t n_leaf;
  int32_t leaf_kind[kMaxLeaves];
  int32_t leaf_obs[kMaxLeaves];
  int32_t leaf_np[kMaxLeaves];
  int32_t leaf_param[kMaxLeaves][kMaxLeafParams];
  int32_t leaf_norm[kMaxLeaves];
  int32_t leaf_root[kMaxLeaves];     // 1: in every term (outside the log-sum-exp)

  int32_t n_term;
  int32_t term_mask[kMaxTerms];      // bit l: leaf l is a factor of term k
  int32_t term_nref[kMaxTerms];
  int32_t term_ref_sum[kMaxTerms][kMaxPathRefs];    // which sum node
  int32_t term_ref_child[kMaxTerms][kMaxPathRefs];  // which coefficient of it

  int32_t n_sum;
  int32_t sum_nchild[kMaxSums];
  int32_t sum_param[kMaxSums][kMaxSumChildren];     // fractions f_1..f_{k-1}, or yields nu_1..nu_k
  int32_t sum_yields[kMaxSums];                     // 1: the sum's coefficients are yields

  int32_t n_acc;                     // accumulators per event stream
  int32_t acc_leaf_base[kMaxLeaves]; // first gradient accumulator of leaf l
  int32_t acc_term_base;             // first term-responsibility accumulator

  int32_t extended;                  // Poisson yield term nu - N ln nu
  int32_t yield_param;               // nu: this parameter, or (-1) the sum of ...
  int32_t ext_sum;                   // ... the yields of this sum (-1: none)
  int32_t want_grad;
  int32_t pad_;
};

// Per-parameter-point constants (device memory / LDS).
struct PerTheta {
  double ec[kMaxLeaves][kLeafConsts];     // per-event constants of each leaf
  double fscale[kMaxLeaves][kMaxLeafParams];  // gradient feature -> d/dtheta scale
  double dlogz[kMaxLeaves][kMaxLeafParams];   // d log Z_l / d theta (local order)
  double logz[kMaxLeaves];                // log Z_l (FP32 pass: log Z_l - kappa_l)
  double ck[kMaxTerms];                   // log w_k - sum log Z over non-root leaves
  double croot;                           // - sum log Z over root leaves
  double dlogw[kMaxTerms][kMaxParams];    // d log w_k / d theta (fraction params)
  double phioff[kMaxLeaves][kMaxLeafParams];  // FP32 pass: feature offsets (else 0)
  int32_t bad;  // bit 0: a parameter outside its range or a leaf's domain; bit 1: a formula leaf's normalisation not positive and finite
  int32_t pad;
};

// Launch schedule of the streaming kernels (picked by the autotuner).
struct Schedule {
  int32_t unroll;          // events per thread per tile iteration
  int32_t blocks_per_cu;   // persistent grid size = CUs * blocks_per_cu
  int32_t tile_events;     // batched mode: events per (set, tile) work item
  int32_t sets_blocks_per_cu;
  int32_t sets_unroll;
};

// Device status bits (accumulated, read back by nll_sync).
enum StatusBits : int32_t { kStatusParam = 1, kStatusPdf = 2 };

}  // namespace nllmi
