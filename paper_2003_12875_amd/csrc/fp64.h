// fp64.h -- double-precision elementary functions for the per-event pass,
// specialised to the argument ranges that occur there, so that they skip
// the special-case handling of the general library routines.
//
// Each is within 2 ulp of the correctly rounded result over its stated
// domain (measured on the device against the host's libm); the likelihood
// needs ~1e-13 relative per event.  Derivation of every constant below:
//   * ln 2 = LN2_HI + LN2_LO, LN2_HI = ln 2 rounded to double;
//   * ln 2 / 256 = LN2_HI / 256 + LN2_LO / 256 (exact scalings);
//   * polynomial coefficients: Chebyshev interpolation (3 resp. 7 points)
//     of the stated function on the stated interval, computed in 50-digit
//     arithmetic and rounded to double.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace nllmi {

constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;

// e^a for a <= 0 (the log-sum-exp factors e^{L_k - m}), by a table:
// a = (256 k + j) ln2/256 + r with integers k,
// j (0 <= j < 256) and |r| <= ln2/512 (n = 256 k + j from one FMA with the
// round-to-integer constant 1.5 * 2^52, whose low word then holds n; each
// reduction step one FMA), e^a = 2^k T_j e^r with T_j = 2^(j/256) from a
// table the kernel keeps in LDS, and e^r - 1 = r + r^2 Q(r), Q the degree-2
// polynomial interpolating (e^r - 1 - r)/r^2 at the 3 Chebyshev points of
// [-ln2/512, ln2/512] (error 0.09 ulp of e^r).  With the table's own
// rounding and the final FMA, measured on the device: at most 1.3 ulp over
// 4.2e6 arguments in [-750, 0], mean error -0.005 ulp.  The argument is
// clamped at -746, where e^a rounds to 0, so that -inf (a term with zero
// density) gives 0.  Per call: 13 VALU instructions and one LDS read (a
// degree-11 polynomial over |r| <= ln2/2 without the table took 18).
constexpr int kExpTabSize = 256;

// T_j for j < kExpTabSize by the device library's exp2, one entry per
// thread of the block at the kernel's start (the caller synchronises the
// block before the first exp_nonpos_tab).
__device__ __forceinline__ void stage_exp_table(double* tab) {
  for (int j = threadIdx.x; j < kExpTabSize; j += blockDim.x) tab[j] = exp2((double)j * (1.0 / kExpTabSize));
}

__device__ __forceinline__ double exp_nonpos_tab(double a, const double* __restrict__ tab) {
  constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52
  a = fmax(a, -746.0);
  const double s = fma(a, 369.3299304675746, kRound);  // 256 / ln 2
  const int n = __double2loint(s);
  const double t = tab[n & (kExpTabSize - 1)];  // issued before the polynomial
  const double nd = s - kRound;
  double r = fma(nd, -kLn2Hi / kExpTabSize, a);
  r = fma(nd, -kLn2Lo / kExpTabSize, r);
  double q = fma(0.04166666857581546, r, 0.16666667812155952);
  q = fma(q, r, 0.5);
  const double p = fma(r * r, q, r);
  return __builtin_ldexp(fma(t, p, t), n >> 8);
}

// ln x for finite x > 0 by a table (the per-event logarithms): x = 2^e m,
// m in [1/2, 1); the top 8 fraction bits of m pick j, the centre c_j of
// m's interval of width 1/512, k_j = 1/c_j rounded to double and
// L_j = -ln k_j (a table the kernel keeps in LDS), so that
// ln m = ln(m k_j) + L_j holds exactly; r = m k_j - 1 from one FMA
// (|r| <= 2^-9), ln(1 + r) = r + r^2 Q(r) with Q the Taylor polynomial of
// degree 4 (truncation below 2e-20), then e ln 2 added with the two-part
// ln 2.  The table's L_j carries the device log's rounding (about 1e-16
// absolute), which is what the likelihood's sums of logarithms need.
// 16 VALU instructions and one LDS read, against ~28 (with a quarter-rate
// reciprocal) for log_pos.
constexpr int kLogTabSize = 256;

// {k_j, L_j} for j < kLogTabSize, one entry per thread of the block at the
// kernel's start (the caller synchronises the block before the first
// log_pos_tab).
__device__ __forceinline__ void stage_log_table(double2* tab) {
  for (int j = threadIdx.x; j < kLogTabSize; j += blockDim.x) {
    const double k = 1.0 / (0.5 + ((double)j + 0.5) * (1.0 / (2 * kLogTabSize)));
    tab[j] = make_double2(k, -log(k));
  }
}

__device__ __forceinline__ double log_pos_tab(double x, const double2* __restrict__ tab) {
  int e;
  const double m = frexp(x, &e);  // m in [1/2, 1)
  const double2 kl = tab[(__double2hiint(m) >> 12) & (kLogTabSize - 1)];
  const double r = fma(m, kl.x, -1.0);
  double q = fma(-0.16666666666666666, r, 0.2);
  q = fma(q, r, -0.25);
  q = fma(q, r, 0.3333333333333333);
  q = fma(q, r, -0.5);
  const double p = fma(r * r, q, r);
  const double ed = (double)e;
  return fma(ed, kLn2Hi, kl.y + fma(ed, kLn2Lo, p));
}

// The per-event logarithms' table: one per block, staged by the kernels
// whose compiled shape takes a logarithm per event.
static __shared__ double2 g_log_tab[kLogTabSize];

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
