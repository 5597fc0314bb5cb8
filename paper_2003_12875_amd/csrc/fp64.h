// fp64.h -- double-precision elementary functions for the per-event pass,
// specialised to the argument ranges that occur there, so that they skip
// the special-case handling of the general library routines.
//
// Each is within 2 ulp of the correctly rounded result over its stated
// domain (measured on the device against the host's libm); the likelihood
// needs ~1e-13 relative per event.  Derivation of every constant below:
//   * ln 2 = LN2_HI + LN2_LO, LN2_HI = ln 2 rounded to double;
//   * polynomial coefficients: Chebyshev interpolation (12 resp. 7 points)
//     of the stated function on the stated interval, computed in 50-digit
//     arithmetic and rounded to double.
#pragma once

#include <hip/hip_runtime.h>

namespace nllmi {

constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;

// e^a for a <= 0 (the log-sum-exp factors e^{L_k - m}).  a = n ln2 + r with
// |r| <= ln2/2 (each reduction step one FMA); e^r by the degree-11
// polynomial interpolating exp at the 12 Chebyshev points of [-ln2/2, ln2/2]
// (interpolation error 3.2e-18 relative, below the rounding of its Horner
// evaluation); then 2^n e^r.  Measured: at most 1 ulp over 4e6 arguments in
// [-750, 0].  The argument is clamped at -746, where e^a rounds to 0, so
// that -inf (a term with zero density) gives 0.
__device__ __forceinline__ double exp_nonpos(double a) {
  a = fmax(a, -746.0);
  const double n = __builtin_rint(a * 1.4426950408889634);
  double r = fma(n, -kLn2Hi, a);
  r = fma(n, -kLn2Lo, r);
  double p = 2.5110037605963777e-08;
  p = fma(p, r, 2.763263963904103e-07);
  p = fma(p, r, 2.755724091857897e-06);
  p = fma(p, r, 2.4801485482328494e-05);
  p = fma(p, r, 0.00019841269890047113);
  p = fma(p, r, 0.0013888888952314775);
  p = fma(p, r, 0.008333333333319601);
  p = fma(p, r, 0.0416666666664881);
  p = fma(p, r, 0.1666666666666668);
  p = fma(p, r, 0.5000000000000019);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return __builtin_ldexp(p, (int)n);
}

// 1/x for the gradient features only (never the likelihood value): the
// hardware reciprocal (2^-24 relative, measured) and one Newton step, 2^-48.
__device__ __forceinline__ double rcp_grad(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// 1/x for finite normal x where the result enters the likelihood value:
// a second Newton step after rcp_grad's takes the 2^-48 error to the
// rounding of the last step (about 1 ulp).
__device__ __forceinline__ double rcp_full(double x) {
  const double r = rcp_grad(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// ln x for finite normal x > 0.  x = 2^e m with m in [sqrt(1/2), sqrt(2));
// ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.1716 (the quotient
// from the refined reciprocal and one residual correction), written as
// 2s + 2s z R(z), z = s^2, R(z) = (atanh(sqrt z) - sqrt z) / sqrt(z)^3
// = 1/3 + z/5 + ... by its degree-6 Chebyshev interpolant on [0, 0.02944]
// (error 1.6e-16 absolute in R, 5e-18 relative in ln m); then e ln 2 added
// with the two-part ln 2.  Emulated: 1.9 ulp at most.
__device__ __forceinline__ double log_pos(double x) {
  int e;
  double m = frexp(x, &e);  // m in [1/2, 1)
  const bool low = m < 0.7071067811865476;
  m = __builtin_ldexp(m, low ? 1 : 0);
  e -= low ? 1 : 0;
  const double f = m - 1.0;  // exact
  const double d = m + 1.0;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  const double s0 = f * r;
  const double s = fma(fma(-s0, d, f), r, s0);
  const double z = s * s;
  double p = 0.07308224842521703;
  p = fma(p, z, 0.07665860800278021);
  p = fma(p, z, 0.09091444562630861);
  p = fma(p, z, 0.1111110556739754);
  p = fma(p, z, 0.14285714312987743);
  p = fma(p, z, 0.19999999999949752);
  p = fma(p, z, 0.3333333333333335);
  const double s2 = s + s;
  const double lm = fma(s2 * z, p, s2);
  const double ed = (double)e;
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, lm));
}

// sqrt x for finite normal x > 0: the hardware reciprocal square root
// refined by one coupled Newton step for (sqrt x, 1/(2 sqrt x)) and a final
// residual correction of sqrt x.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

}  // namespace nllmi
