// fp32.h -- single-precision building blocks of the FP32-compensated event
// pass (the precision mode in which the per-event density arithmetic runs
// in FP32 while normalisation, reductions across threads and the minimiser
// stay in FP64).
//
// The NLL is a sum over up to ~1e8 events, so a per-event error that is
// random (unbiased rounding) averages out as sqrt(N) while a systematic one
// grows as N.  Everything here is therefore built from IEEE round-to-nearest
// additions, multiplications and FMAs (unbiased), with polynomial
// truncation errors kept near 1e-9 relative; the hardware approximations
// (v_exp_f32, v_log_f32, v_rcp_f32, v_sqrt_f32) are used only as starting
// values that one Newton step then corrects.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace nllmi {

// a double as an unevaluated float sum hi + lo (|lo| <= ulp(hi)/2)
struct F2 {
  float hi, lo;
};
__device__ inline F2 split2(double v) {
  const float hi = (float)v;
  return F2{hi, (float)(v - (double)hi)};
}
// x * (hi + lo), the product of a float with a split constant
__device__ inline float mul2(float x, F2 c) { return fmaf(x, c.hi, x * c.lo); }
// x * c + d for split c and d
__device__ inline float fma2(float x, F2 c, F2 d) { return fmaf(x, c.hi, d.hi) + fmaf(x, c.lo, d.lo); }

// 1/s: hardware reciprocal plus one Newton step
__device__ inline float rcp_f32(float s) {
  const float r = __builtin_amdgcn_rcpf(s);
  return fmaf(r, fmaf(-s, r, 1.0f), r);
}

// sqrt(u), u >= 0: hardware square root plus one Newton step on the residual
__device__ inline float sqrt_f32(float u) {
  const float s = __builtin_sqrtf(u);
  if (!(s > 0.0f)) return s;
  const float e = fmaf(-s, s, u);
  return fmaf(e, 0.5f * __builtin_amdgcn_rcpf(s), s);
}

// e^d for d <= ~88: d = k ln2 + f with Cody-Waite reduction (ln2 split so
// that k * LN2_HI is exact for |k| < 2^8), e^f by its Taylor polynomial of
// degree 8 on |f| <= ln2 / 2 (truncation below 2.1e-10 relative), 2^k by
// ldexp.  Underflows to 0 for d < -103.
__device__ inline float exp_f32(float d) {
  constexpr float kLog2e = 1.44269504088896341f;
  constexpr float kLn2Hi = 0.693145751953125f;    // 0x3f317200
  constexpr float kLn2Lo = 1.4286068203094172e-06f;
  const float dk = d < -104.0f ? -104.0f : d;  // NaN propagates
  const float k = __builtin_rintf(dk * kLog2e);
  float f = fmaf(-k, kLn2Hi, dk);
  f = fmaf(-k, kLn2Lo, f);
  float p = 2.48015873015873e-05f;                // 1/8!
  p = fmaf(p, f, 1.98412698412698e-04f);          // 1/7!
  p = fmaf(p, f, 1.38888888888889e-03f);          // 1/6!
  p = fmaf(p, f, 8.33333333333333e-03f);          // 1/5!
  p = fmaf(p, f, 4.16666666666667e-02f);          // 1/4!
  p = fmaf(p, f, 1.66666666666667e-01f);          // 1/3!
  p = fmaf(p, f, 0.5f);
  p = fmaf(p, f, 1.0f);
  p = fmaf(p, f, 1.0f);
  return __builtin_ldexpf(p, (int)k);
}

// log(D) for finite D > 0: D = 2^e m with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(z), z = (m - 1)/(m + 1), |z| <= 0.1716, by its odd series
// through z^11 (truncation below 2e-10 absolute); e ln2 with a split ln2.
// Returns -inf for D = 0 and NaN for D < 0.
__device__ inline float log_f32(float D) {
  constexpr float kLn2Hi = 0.693145751953125f;
  constexpr float kLn2Lo = 1.4286068203094172e-06f;
  if (!(D > 0.0f) || D == __builtin_inff()) return D == 0.0f ? -__builtin_inff() : (D > 0.0f ? D : __builtin_nanf(""));
  int e = __builtin_amdgcn_frexp_expf(D);
  float m = __builtin_amdgcn_frexp_mantf(D);  // [0.5, 1)
  if (m < 0.70710678f) {
    m += m;
    e -= 1;
  }
  const float num = m - 1.0f;  // exact
  const float den = m + 1.0f;
  const float r = rcp_f32(den);
  float z = num * r;
  z = fmaf(r, fmaf(-z, den, num), z);  // one correction of the quotient
  const float z2 = z * z;
  float p = 1.0f / 11.0f;
  p = fmaf(p, z2, 1.0f / 9.0f);
  p = fmaf(p, z2, 1.0f / 7.0f);
  p = fmaf(p, z2, 1.0f / 5.0f);
  p = fmaf(p, z2, 1.0f / 3.0f);
  const float lm = fmaf(2.0f * z * z2, p, 2.0f * z);
  const float fe = (float)e;
  return fmaf(fe, kLn2Hi, fmaf(fe, kLn2Lo, lm));
}

// Knuth's TwoSum: s + err == a + b exactly
__device__ inline void two_sum(float a, float b, float& s, float& err) {
  s = a + b;
  const float bb = s - a;
  err = (a - (s - bb)) + (b - bb);
}

}  // namespace nllmi
