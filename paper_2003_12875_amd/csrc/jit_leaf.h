// jit_leaf.h -- a density given as a formula string (Sec. 4: PDFs written
// as expressions and compiled at run time) as one leaf of a composite
// model, beside the built-in leaves: sums and products of it with any
// other leaf go through the same kernels as every other shape.
//
// F is generated at model creation from the formula (rtc.cpp) and compiled
// together with these templates by hipRTC:
//   struct F {
//     template <int N> using D = <forward-mode dual number over N parameters>;
//     static double val(double x, const double* p);         // g(x; p)
//     template <int N> static D<N> dual(double x, const D<N>* p);
//   };
// The dual type carries the value .v and the derivatives .d[k] through
// every operation, so that one evaluation gives g and dg/dp_k.
//
// Per event: lambda = log g (the staged logarithm table; g = 0 gives -inf,
// a term that contributes nothing; g < 0 or non-finite makes the
// likelihood non-finite, reported as an invalid density) and the features
// phi_k = (dg/dp_k) / g, which the model multiplies by the term's
// responsibility (0 where g = 0, and so are the features; a subnormal g is
// scaled by 2^64 before its reciprocal, which would otherwise overflow and
// meet a responsibility of 0 as inf x 0).
// Normalisation: composite 256-point Gauss-Legendre over [lo, hi] on 1, 2,
// 4, ... kJitMaxPanels equal panels, until two successive levels agree
// (compute_pertheta, phase 1, with norm_level below for one thread's nodes).
#pragma once

#include "plan.h"

namespace nllmi {

template <int NP_, class F>
struct JitLeaf {
  static_assert(NP_ >= 1 && NP_ <= kJitMaxLeafParams, "formula leaf parameters");
  static constexpr int kKind = kJit;
  static constexpr int NP = NP_;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = true;   // a logarithm per event
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = true;    // adaptive composite Gauss-Legendre (norm_level)
  static constexpr int kSetupLanes = 1;
  using DT = typename F::template D<NP_>;
  struct C {
    double p[NP_];
  };
  struct C32 {};  // no FP32-compensated pass for this leaf
  __device__ static bool valid(const double*) { return true; }  // the formula's own domain decides, per event
  // the parameters themselves are the event constants; the features are
  // d log g / d p_k directly (scale 1); Z comes from the numerical rule
  __device__ static void setup(const double* p, double, double, bool, LeafSetup& s) {
#pragma unroll
    for (int j = 0; j < NP_; ++j) {
      s.ec[j] = p[j];
      s.fscale[j] = 1.0;
    }
  }
  __device__ static C load(const double* ec) {
    C c;
#pragma unroll
    for (int j = 0; j < NP_; ++j) c.p[j] = ec[j];
    return c;
  }
  // the parameters as independent dual variables
  __device__ static void seed(const double* p, DT (&pd)[NP_]) {
#pragma unroll
    for (int j = 0; j < NP_; ++j) {
      pd[j].v = p[j];
#pragma unroll
      for (int k = 0; k < NP_; ++k) pd[j].d[k] = j == k ? 1.0 : 0.0;
    }
  }
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    gam = 1.0;
    if constexpr (GRAD) {
      DT pd[NP_];
      seed(c.p, pd);
      const DT g = F::template dual<NP_>(x, pd);
      lam = log_g(g.v);
      // without a branch: g'_k s times the refined reciprocal of g s, s = 2^64
      // for subnormal g (g s is then exact and normal), else 1
      const double s = g.v < 2.2250738585072014e-308 ? 18446744073709551616.0 : 1.0;
      const double r = rcp_grad(g.v * s);
      const bool pos = g.v > 0.0;
#pragma unroll
      for (int k = 0; k < NP_; ++k) phi[k] = pos ? (g.d[k] * s) * r : 0.0;
    } else {
      lam = log_g(F::val(x, c.p));
    }
  }
  // log g by the staged table for positive finite g; the logarithm's own
  // values otherwise (-inf at 0, +inf at +inf, NaN below 0 or at NaN),
  // selected as constants so that no second logarithm is evaluated
  __device__ static inline double log_g(double g) {
    const bool fin = g > 0.0 && g <= 1.7976931348623157e308;
    const double lt = log_pos_tab(fin ? g : 1.0, g_log_tab);
    const double inv = g == 0.0 ? -__builtin_inf() : (g > 0.0 ? __builtin_inf() : __builtin_nan(""));
    return fin ? lt : inv;
  }
  // This thread's share of the composite rule on n_pan equal panels of
  // [lo, hi]: node t of every panel (t < 256), with w g and w dg/dp_k
  // summed into z and w |g|, w |dg/dp_k| into ab (the error scales of the
  // agreement test).  The last panel ends exactly at hi.
  __device__ static void norm_level(const double* p, double lo, double hi, int n_pan, const double* glx,
                                    const double* glw, int t, double (&z)[NP_ + 1], double (&ab)[NP_ + 1]) {
#pragma unroll
    for (int k = 0; k <= NP_; ++k) z[k] = ab[k] = 0.0;
    DT pd[NP_];
    seed(p, pd);
    const double H = (hi - lo) / n_pan, h = 0.5 * H;
    const double w = h * glw[t], xt = glx[t];
    for (int j = 0; j < n_pan; ++j) {
      const double x = j + 1 == n_pan ? fma(h, xt, hi - h) : fma(h, xt, fma((double)j, H, lo + h));
      const DT g = F::template dual<NP_>(x, pd);
      z[0] += w * g.v;
      ab[0] += w * fabs(g.v);
#pragma unroll
      for (int k = 0; k < NP_; ++k) {
        z[1 + k] += w * g.d[k];
        ab[1 + k] += w * fabs(g.d[k]);
      }
    }
  }
};

}  // namespace nllmi
