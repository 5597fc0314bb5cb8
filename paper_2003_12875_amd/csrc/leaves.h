// leaves.h -- the built-in leaf densities on the device (gfx950).
//
// Each leaf type provides
//   * setup():   per-parameter-point constants for the event pass, the
//                normalisation integral Z and dZ/dtheta (closed form), and
//                the scale that maps each gradient feature to d log g/dtheta;
//   * shape():   the unnormalised density and its parameter derivatives at
//                one point (for Gauss-Legendre normalisation);
//   * event():   the per-event part, fused into the single streaming pass.
//                It returns lam (log-domain part of log g), gam (a linear
//                factor, 1 for pure log-domain leaves: used when the leaf is
//                a root factor so that no per-event log is needed) and the
//                gradient features phi_p with d log g / d theta_p =
//                fscale_p * phi_p.
//
// The densities are the ones of the paper's built-in models (Sec. 3):
//   Gauss(mu, sigma)        g = exp(-t^2/2),        t = (x - mu)/sigma
//   Exp(c)                  g = exp(c x)
//   Cheb(a_1..a_K)          g = 1 + sum a_k T_k(x'), x' mapped to [-1, 1]
//   CrystalBall(m0,s,a,n)   g = exp(-t^2/2) for t > -a, A (B - t)^-n below,
//                           A = (n/a)^n e^{-a^2/2}, B = n/a - a
//   Argus(m0, c)            g = m sqrt(u) e^{c u}, u = 1 - (m/m0)^2, m < m0
//   Johnson(mu,lam,gam,del) g = e^{-u^2/2} / sqrt(1 + z^2), z = (x - mu)/lam,
//                           u = gam + del asinh(z)   (Johnson's S_U family)
//   ChiSquare(nu)           g = x^{nu/2 - 1} e^{-x/2}, 0 <= x
// Selects are branch-free (both sides computed, one kept, as in Sec. 5.3)
// where both sides are cheap; the Crystal Ball's rare power-law tail is a
// real branch, which a 64-lane wavefront skips when none of its events is
// in the tail.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "fp32.h"
#include "fp64.h"
#include "plan.h"

namespace nllmi {

constexpr double kSqrtPiOver2 = 1.2533141373155002512078826424055;  // sqrt(pi/2)
constexpr double kSqrtPi = 1.7724538509055160272981674833411;
constexpr double kInvSqrt2 = 0.70710678118654752440084436210485;
constexpr double kLn2 = 0.69314718055994530941723212145818;

// erf(b/sqrt2) - erf(a/sqrt2) for a <= b without cancellation in the tails
__device__ inline double erf_span(double a, double b) {
  if (a >= 0.0) return erfc(a * kInvSqrt2) - erfc(b * kInvSqrt2);
  if (b <= 0.0) return erfc(-b * kInvSqrt2) - erfc(-a * kInvSqrt2);
  return erf(b * kInvSqrt2) - erf(a * kInvSqrt2);
}

// Closed-form pieces are written for the leaf's local parameter order.
// kappa and phioff serve the FP32 event pass only, where a leaf may work on
// x - x0 for a location x0: its log-density then differs by the constant
// kappa (added to the term constants in FP64) and feature p by phioff[p]
// (restored in FP64 after the reduction).
struct LeafSetup {
  double ec[kLeafConsts];  // event constants
  double fscale[kMaxLeafParams];
  double Z;
  double dZ[kMaxLeafParams];
  double kappa;
  double phioff[kMaxLeafParams];
};

// ------------------------------------------------------------------------
// Gaussian
// ------------------------------------------------------------------------
struct GaussLeaf {
  static constexpr int kKind = kGauss;
  static constexpr int NP = 2;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = false;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  struct C {
    double is, b;
  };
  __device__ static bool valid(const double* p) { return p[1] > 0.0; }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    const double mu = p[0], sg = p[1], is = 1.0 / sg;
    s.ec[0] = is;
    s.ec[1] = -mu * is;
    s.ec[2] = mu;
    s.fscale[0] = is;
    s.fscale[1] = is;
    if (!analytic) return;
    const double a = (lo - mu) * is, b = (hi - mu) * is;
    const double ea = exp(-0.5 * a * a), eb = exp(-0.5 * b * b);
    s.Z = sg * kSqrtPiOver2 * erf_span(a, b);
    s.dZ[0] = ea - eb;
    s.dZ[1] = s.Z * is + a * ea - b * eb;
  }
  // setup() over 4 lanes of one wave (lane 0 = the group's first): the two
  // error-function values of erf_span and the two boundary exponentials each
  // on a lane of their own, gathered by shuffles; the same operations as
  // setup(), so the same bits.  The result is complete on lane 0.
  static constexpr int kSetupLanes = 4;
  __device__ static void setup_coop(const double* p, double lo, double hi, bool analytic, LeafSetup& s, int lane) {
    const double mu = p[0], sg = p[1], is = 1.0 / sg;
    s.ec[0] = is;
    s.ec[1] = -mu * is;
    s.ec[2] = mu;
    s.fscale[0] = is;
    s.fscale[1] = is;
    if (!analytic) return;
    const double a = (lo - mu) * is, b = (hi - mu) * is;
    double v;
    if (lane >= 2) {
      const double t = lane == 2 ? a : b;
      v = exp(-0.5 * t * t);
    } else if (a >= 0.0) {  // erf_span = v(lane 0) - v(lane 1)
      v = erfc((lane ? b : a) * kInvSqrt2);
    } else if (b <= 0.0) {
      v = erfc((lane ? -a : -b) * kInvSqrt2);
    } else {
      v = erf((lane ? a : b) * kInvSqrt2);
    }
    const int base = (int)(threadIdx.x & 63) - lane;
    const double u0 = __shfl(v, base, 64), u1 = __shfl(v, base + 1, 64);
    const double ea = __shfl(v, base + 2, 64), eb = __shfl(v, base + 3, 64);
    s.Z = sg * kSqrtPiOver2 * (u0 - u1);
    s.dZ[0] = ea - eb;
    s.dZ[1] = s.Z * is + a * ea - b * eb;
  }
  __device__ static double shape(const double* p, double lo, double hi, double x, double* dg) {
    const double t = (x - p[0]) / p[1];
    const double g = exp(-0.5 * t * t);
    dg[0] = g * t / p[1];
    dg[1] = g * t * t / p[1];
    return g;
  }
  __device__ static C load(const double* ec) { return C{ec[0], ec[1]}; }
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double t = fma(x, c.is, c.b);
    const double tt = t * t;
    lam = -0.5 * tt;
    gam = 1.0;
    if (GRAD) {
      phi[0] = t;
      phi[1] = tt;
    }
  }
  // FP32 pass: x - mu in FP64, then single precision
  struct C32 {
    double mu;
    F2 is;
  };
  __device__ static C32 load32(const double* ec) { return C32{ec[2], split2(ec[0])}; }
  template <bool GRAD>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float t = mul2((float)(x - c.mu), c.is);
    const float tt = t * t;
    lam = -0.5f * tt;
    gam = 1.0f;
    if (GRAD) {
      phi[0] = t;
      phi[1] = tt;
    }
  }
};

// ------------------------------------------------------------------------
// Exponential
// ------------------------------------------------------------------------
struct ExpLeaf {
  static constexpr int kKind = kExp;
  static constexpr int NP = 1;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = false;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  struct C {
    double c;
  };
  __device__ static bool valid(const double*) { return true; }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    const double c = p[0];
    const double x0 = 0.5 * (lo + hi);  // FP32 pass: location of x
    s.ec[0] = c;
    s.ec[1] = x0;
    s.fscale[0] = 1.0;
    s.kappa = c * x0;
    s.phioff[0] = x0;
    if (!analytic) return;
    const double R = fmax(fabs(lo), fabs(hi));
    if (fabs(c) * R < 0.25) {
      // int x^j e^{cx} as a power series in c (all terms small)
      double z = 0.0, dz = 0.0, ck = 1.0, hp = hi, lp = lo;
      for (int k = 0; k < 40; ++k) {
        z += ck * (hp - lp) / (k + 1);
        dz += ck * (hp * hi - lp * lo) / (k + 2);
        hp *= hi;
        lp *= lo;
        ck *= c / (k + 1);
      }
      s.Z = z;
      s.dZ[0] = dz;
      return;
    }
    const double elo = exp(c * lo), ehi = exp(c * hi);
    s.Z = elo * expm1(c * (hi - lo)) / c;
    s.dZ[0] = (ehi * fma(c, hi, -1.0) - elo * fma(c, lo, -1.0)) / (c * c);
  }
  // setup() over 3 lanes: exp(c lo), exp(c hi) and expm1(c (hi - lo)) each
  // on a lane of their own (same operations, same bits); complete on lane 0.
  static constexpr int kSetupLanes = 3;
  __device__ static void setup_coop(const double* p, double lo, double hi, bool analytic, LeafSetup& s, int lane) {
    const double c = p[0];
    const double R = fmax(fabs(lo), fabs(hi));
    if (!analytic || fabs(c) * R < 0.25) {  // no transcendental functions to spread
      setup(p, lo, hi, analytic, s);
      return;
    }
    const double x0 = 0.5 * (lo + hi);
    s.ec[0] = c;
    s.ec[1] = x0;
    s.fscale[0] = 1.0;
    s.kappa = c * x0;
    s.phioff[0] = x0;
    double v;
    if (lane == 0) {
      v = expm1(c * (hi - lo));
    } else {
      v = exp(c * (lane == 1 ? lo : hi));
    }
    const int base = (int)(threadIdx.x & 63) - lane;
    const double em = __shfl(v, base, 64), elo = __shfl(v, base + 1, 64), ehi = __shfl(v, base + 2, 64);
    s.Z = elo * em / c;
    s.dZ[0] = (ehi * fma(c, hi, -1.0) - elo * fma(c, lo, -1.0)) / (c * c);
  }
  __device__ static double shape(const double* p, double, double, double x, double* dg) {
    const double g = exp(p[0] * x);
    dg[0] = g * x;
    return g;
  }
  __device__ static C load(const double* ec) { return C{ec[0]}; }
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    lam = c.c * x;
    gam = 1.0;
    if (GRAD) phi[0] = x;
  }
  // FP32 pass on x' = x - x0: c x = c x' + kappa, feature x = x' + phioff
  struct C32 {
    double x0;
    F2 c;
  };
  __device__ static C32 load32(const double* ec) { return C32{ec[1], split2(ec[0])}; }
  template <bool GRAD>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float xp = (float)(x - c.x0);
    lam = mul2(xp, c.c);
    gam = 1.0f;
    if (GRAD) phi[0] = xp;
  }
};

// ------------------------------------------------------------------------
// Chebyshev series of order K (T_0 coefficient 1); linear when a root factor
// ------------------------------------------------------------------------
template <int K>
struct ChebLeaf {
  static_assert(K >= 1 && K <= 8, "Chebyshev order 1..8");
  static constexpr int kKind = kCheb;
  static constexpr int NP = K;
  static constexpr bool kLinear = true;
  static constexpr bool kEventLog = false;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  static constexpr int kSetupLanes = 1;  // setup() on one lane
  struct C {
    double sx, ox, a[K];
  };
  __device__ static bool valid(const double*) { return true; }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    s.ec[0] = 2.0 / (hi - lo);
    s.ec[1] = -(hi + lo) / (hi - lo);
    for (int k = 0; k < K; ++k) {
      s.ec[2 + k] = p[k];
      s.fscale[k] = 1.0;
    }
    if (!analytic) return;
    // int_{-1}^{1} T_k dx' = 2/(1-k^2) (k even), 0 (k odd); dx = (hi-lo)/2 dx'
    const double half = 0.5 * (hi - lo);
    double z = 2.0 * half;
    for (int k = 1; k <= K; ++k) {
      const double w = (k & 1) ? 0.0 : 2.0 / (1.0 - (double)(k * k));
      z += half * p[k - 1] * w;
      s.dZ[k - 1] = half * w;
    }
    s.Z = z;
  }
  __device__ static double shape(const double* p, double lo, double hi, double x, double* dg) {
    const double y = (2.0 * x - lo - hi) / (hi - lo);
    double t0 = 1.0, t1 = y, g = 1.0;
    for (int k = 0; k < K; ++k) {
      g += p[k] * t1;
      dg[k] = t1;
      const double t2 = 2.0 * y * t1 - t0;
      t0 = t1;
      t1 = t2;
    }
    return g;
  }
  __device__ static C load(const double* ec) {
    C c;
    c.sx = ec[0];
    c.ox = ec[1];
    for (int k = 0; k < K; ++k) c.a[k] = ec[2 + k];
    return c;
  }
  // LIN: leave g as a linear factor (root factor) instead of taking its log.
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double y = fma(x, c.sx, c.ox);
    const double y2 = y + y;
    double tk[K];
    double tm = 1.0, t = y;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      tk[k] = t;
      const double tn = fma(y2, t, -tm);
      tm = t;
      t = tn;
    }
    double g = 1.0;
#pragma unroll
    for (int k = 0; k < K; ++k) g = fma(c.a[k], tk[k], g);
    if (LIN) {
      lam = 0.0;
      gam = g;
    } else {
      lam = log(g);
      gam = 1.0;
    }
    if (GRAD) {
      const double r = rcp_grad(g);
#pragma unroll
      for (int k = 0; k < K; ++k) phi[k] = tk[k] * r;
    }
  }
  // FP32 pass: the mapped coordinate in FP64, the polynomials T_k in
  // single precision, their combination with the coefficients in FP64 (a
  // per-point constant added to a single-precision value would always
  // lose the same low bits), the logarithm and reciprocal in single
  // precision.
  struct C32 {
    double sx, ox;
    double a[K];
  };
  __device__ static C32 load32(const double* ec) {
    C32 c;
    c.sx = ec[0];
    c.ox = ec[1];
    for (int k = 0; k < K; ++k) c.a[k] = ec[2 + k];
    return c;
  }
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float y = (float)fma(x, c.sx, c.ox);
    const float y2 = y + y;
    float tk[K];
    float tm = 1.0f, t = y;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      tk[k] = t;
      const float tn = fmaf(y2, t, -tm);
      tm = t;
      t = tn;
    }
    double g64 = 1.0;
#pragma unroll
    for (int k = 0; k < K; ++k) g64 = fma(c.a[k], (double)tk[k], g64);
    const float g = (float)g64;
    if (LIN) {
      lam = 0.0f;
      gam = g;
    } else {
      lam = log_f32(g);
      gam = 1.0f;
    }
    if (GRAD) {
      const float r = rcp_f32(g);
#pragma unroll
      for (int k = 0; k < K; ++k) phi[k] = tk[k] * r;
    }
  }
};

// ------------------------------------------------------------------------
// Crystal Ball (low-side tail)
// ------------------------------------------------------------------------
struct CBLeaf {
  static constexpr int kKind = kCB;
  static constexpr int NP = 4;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = true;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  static constexpr int kSetupLanes = 1;  // setup() on one lane
  struct C {
    double is, b, na, logA, B, n, Ka, Kb, Kc, nOverA;
  };
  __device__ static bool valid(const double* p) { return p[1] > 0.0 && p[2] > 0.0 && p[3] > 1.0; }

  // closed-form integral over t in [ca, cb] of the core and [ta, tb] of the tail
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    const double m0 = p[0], sg = p[1], al = p[2], n = p[3], is = 1.0 / sg;
    const double logA = n * log(n / al) - 0.5 * al * al;
    const double B = n / al - al;
    s.ec[0] = is;
    s.ec[1] = -m0 * is;
    s.ec[2] = -al;
    s.ec[3] = logA;
    s.ec[4] = B;
    s.ec[5] = n;
    s.ec[6] = -n / al - al;                 // d log A/d alpha
    s.ec[7] = n * (n / (al * al) + 1.0);    // -n dB/d alpha
    s.ec[8] = log(n / al) + 1.0;            // d log A / d n
    s.ec[9] = n / al;                       // n dB/dn
    s.ec[10] = m0;                          // FP32 pass: location
    s.fscale[0] = is;
    s.fscale[1] = is;
    s.fscale[2] = 1.0;
    s.fscale[3] = 1.0;
    if (!analytic) return;
    const double tlo = (lo - m0) * is, thi = (hi - m0) * is;
    double Z = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    const double ca = fmax(tlo, -al), cb = thi;
    if (cb > ca) {
      const double ea = exp(-0.5 * ca * ca), eb = exp(-0.5 * cb * cb);
      const double zc = sg * kSqrtPiOver2 * erf_span(ca, cb);
      Z += zc;
      d0 += ea - eb;                       // int t e^{-t^2/2} dt
      d1 += zc * is + ca * ea - cb * eb;   // int t^2 e^{-t^2/2} dt
    }
    const double ta = tlo, tb = fmin(thi, -al);
    if (tb > ta) {
      const double A = exp(logA);
      const double Da = B - ta, Db = B - tb;  // Db < Da
      const double lDa = log(Da), lDb = log(Db);
      const double pa = exp(-n * lDa), pb = exp(-n * lDb);         // D^-n
      const double qa = Da * pa, qb = Db * pb;                     // D^{1-n}
      const double n1 = n - 1.0;
      const double I0 = (qb - qa) / n1;        // int D^-n dt
      const double I1 = (pb - pa) / n;         // int D^{-n-1} dt
      // int D^-n ln D dt = [D^{1-n} (ln D/(n-1) + 1/(n-1)^2)]
      const double IL = qb * (lDb / n1 + 1.0 / (n1 * n1)) - qa * (lDa / n1 + 1.0 / (n1 * n1));
      const double zt = sg * A * I0;
      Z += zt;
      d0 += -n * A * I1;                                // m0
      d1 += -n * A * (B * I1 - I0);                     // sigma: t = B - D
      d2 += s.ec[6] * zt + s.ec[7] * sg * A * I1;       // alpha
      d3 += s.ec[8] * zt - sg * A * IL - s.ec[9] * sg * A * I1;  // n
    }
    s.Z = Z;
    s.dZ[0] = d0;
    s.dZ[1] = d1;
    s.dZ[2] = d2;
    s.dZ[3] = d3;
  }
  __device__ static double shape(const double* p, double lo, double hi, double x, double* dg) {
    const double m0 = p[0], sg = p[1], al = p[2], n = p[3];
    const double t = (x - m0) / sg;
    if (t > -al) {
      const double g = exp(-0.5 * t * t);
      dg[0] = g * t / sg;
      dg[1] = g * t * t / sg;
      dg[2] = 0.0;
      dg[3] = 0.0;
      return g;
    }
    const double B = n / al - al, D = B - t;
    const double g = exp(n * log(n / al) - 0.5 * al * al - n * log(D));
    dg[0] = -g * n / (sg * D);
    dg[1] = -g * n * t / (sg * D);
    dg[2] = g * (-n / al - al + n * (n / (al * al) + 1.0) / D);
    dg[3] = g * (log(n / al) + 1.0 - log(D) - n / (al * D));
    return g;
  }
  __device__ static C load(const double* ec) {
    return C{ec[0], ec[1], ec[2], ec[3], ec[4], ec[5], ec[6], ec[7], ec[8], ec[9]};
  }
  // The power-law tail is a real branch (a wavefront skips it unless one of
  // its lanes is in the tail), the core a straight line.  In a mixture every
  // event evaluates the Crystal Ball, so events of the other components
  // below the junction take the tail too.
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double t = fma(x, c.is, c.b);
    const double tt = t * t;
    lam = -0.5 * tt;
    gam = 1.0;
    if (GRAD) {
      phi[0] = t;
      phi[1] = tt;
      phi[2] = 0.0;
      phi[3] = 0.0;
    }
    if (!(t > c.na)) {
      const double D = c.B - t;  // >= n / alpha > 0
      const double lD = log_pos_tab(D, g_log_tab);
      lam = fma(-c.n, lD, c.logA);
      if (GRAD) {
        const double r = rcp_grad(D);
        const double nr = c.n * r;
        phi[0] = -nr;
        phi[1] = -nr * t;
        phi[2] = fma(c.Kb, r, c.Ka);
        phi[3] = (c.Kc - lD) - c.nOverA * r;
      }
    }
  }
  // FP32 pass: x - m0 in FP64, t, the logarithm and reciprocal in single
  // precision; the steps that add per-point constants (B - t, log A - n log D
  // and the alpha / n features) in FP64.
  struct C32 {
    double m0, logA, B, n, Ka, Kb, Kc, nOverA;
    F2 is;
    float na;
  };
  __device__ static C32 load32(const double* ec) {
    C32 c;
    c.m0 = ec[10];
    c.is = split2(ec[0]);
    c.na = (float)ec[2];
    c.logA = ec[3];
    c.B = ec[4];
    c.n = ec[5];
    c.Ka = ec[6];
    c.Kb = ec[7];
    c.Kc = ec[8];
    c.nOverA = ec[9];
    return c;
  }
  template <bool GRAD>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float t = mul2((float)(x - c.m0), c.is);
    const float tt = t * t;
    lam = -0.5f * tt;
    gam = 1.0f;
    if (GRAD) {
      phi[0] = t;
      phi[1] = tt;
      phi[2] = 0.0f;
      phi[3] = 0.0f;
    }
    if (!(t > c.na)) {  // the tail, a real branch as in the FP64 pass
      const double D64 = c.B - (double)t;
      const float D = (float)D64;
      const float r = rcp_f32(D);
      // log D to first order in the rounding of D
      const double lD = (double)log_f32(D) + (D64 - (double)D) * (double)r;
      lam = (float)fma(-c.n, lD, c.logA);
      if (GRAD) {
        const float nr = (float)(c.n * (double)r);
        phi[0] = -nr;
        phi[1] = -nr * t;
        phi[2] = (float)fma(c.Kb, (double)r, c.Ka);
        phi[3] = (float)((c.Kc - lD) - c.nOverA * (double)r);
      }
    }
  }
};

// ------------------------------------------------------------------------
// ARGUS (power 1/2)
// ------------------------------------------------------------------------
// J_p(U) = int_0^U u^p e^{c u} du for p in {-1/2, 1/2, 3/2}, through the
// lower incomplete gamma function gamma(p+1, kU)/k^{p+1} (k = -c > 0):
//   gamma(1/2, z) = sqrt(pi) erf(sqrt z)
//   gamma(a+1, z) = a gamma(a, z) - z^a e^{-z}
// with the series gamma(a, z) = z^a sum_j (-z)^j / (j! (a + j)) for z < 1
// (where the recurrence cancels); c >= 0 uses the power series of e^{cu}.
__device__ inline void argus_J(double c, double U, double J[3]) {
  J[0] = J[1] = J[2] = 0.0;
  if (!(U > 0.0)) return;
  const double ap[3] = {0.5, 1.5, 2.5};
  if (c >= 0.0) {
    const double x = c * U;
    for (int q = 0; q < 3; ++q) {
      double sum = 0.0, term = 1.0;
      for (int j = 0; j < 400; ++j) {
        const double add = term / (j + ap[q]);
        sum += add;
        if (add < 1e-18 * sum) break;
        term *= x / (j + 1);
      }
      J[q] = pow(U, ap[q]) * sum;
    }
    return;
  }
  const double k = -c, z = k * U;
  double g[3];
  if (z < 1.0) {
    for (int q = 0; q < 3; ++q) {
      double sum = 0.0, term = 1.0;
      for (int j = 0; j < 60; ++j) {
        sum += term / (j + ap[q]);
        term *= -z / (j + 1);
      }
      g[q] = pow(z, ap[q]) * sum;
    }
  } else {
    const double sz = sqrt(z), ez = exp(-z);
    g[0] = kSqrtPi * erf(sz);
    g[1] = 0.5 * g[0] - sz * ez;
    g[2] = 1.5 * g[1] - z * sz * ez;
  }
  for (int q = 0; q < 3; ++q) J[q] = g[q] / pow(k, ap[q]);
}

struct ArgusLeaf {
  static constexpr int kKind = kArgus;
  static constexpr int NP = 2;
  static constexpr bool kLinear = true;
  static constexpr bool kEventLog = false;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  static constexpr int kSetupLanes = 1;  // setup() on one lane
  struct C {
    double m0, im02, c, dm0;  // dm0: 2/m0^3, or 0 when m0 is not differentiated
  };
  __device__ static bool valid(const double* p) { return true; }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    const double m0 = p[0], c = p[1];
    s.ec[0] = m0;
    s.ec[1] = 1.0 / (m0 * m0);
    s.ec[2] = c;
    s.ec[3] = 2.0 / (m0 * m0 * m0);
    s.fscale[0] = 1.0;
    s.fscale[1] = 1.0;
    if (!analytic) return;
    const double Ua = (m0 - lo) * (m0 + lo) / (m0 * m0);
    const double Ub = hi >= m0 ? 0.0 : (m0 - hi) * (m0 + hi) / (m0 * m0);
    double Ja[3], Jb[3];
    argus_J(c, Ua, Ja);
    argus_J(c, Ub, Jb);
    const double jm = Ja[0] - Jb[0], j1 = Ja[1] - Jb[1], j3 = Ja[2] - Jb[2];
    s.Z = 0.5 * m0 * m0 * j1;
    s.dZ[0] = m0 * (0.5 * (jm - j1) + c * (j1 - j3));
    s.dZ[1] = 0.5 * m0 * m0 * j3;
  }
  __device__ static double shape(const double* p, double, double, double x, double* dg) {
    const double m0 = p[0], c = p[1];
    if (x >= m0) {
      dg[0] = dg[1] = 0.0;
      return 0.0;
    }
    const double u = (m0 - x) * (m0 + x) / (m0 * m0);
    const double g = x * sqrt(u) * exp(c * u);
    dg[0] = g * (0.5 / u + c) * 2.0 * x * x / (m0 * m0 * m0);
    dg[1] = g * u;
    return g;
  }
  // the integrand after m = m0 - s^2 (analytic in s), times dm/ds = 2 s
  __device__ static double shape_subst(const double* p, double sv, double* dg) {
    const double m0 = p[0], c = p[1];
    const double s2 = sv * sv, m = m0 - s2;
    const double u = s2 * (2.0 * m0 - s2) / (m0 * m0);
    const double g = m * sqrt(u) * exp(c * u) * 2.0 * sv;
    dg[0] = g * (0.5 / u + c) * 2.0 * m * m / (m0 * m0 * m0);
    dg[1] = g * u;
    return g;
  }
  __device__ static C load(const double* ec) { return C{ec[0], ec[1], ec[2], ec[3]}; }
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double u = (c.m0 - x) * (c.m0 + x) * c.im02;
    const bool in = u > 0.0;
    const double us = in ? u : 1.0;
    if (LIN) {
      lam = in ? c.c * us : -__builtin_inf();
      gam = in ? x * sqrt_pos(us) : 0.0;  // us: u > 0 (normal) or 1
    } else {
      lam = in ? fma(0.5, log(x * x * us), c.c * us) : -__builtin_inf();
      gam = 1.0;
    }
    if (GRAD) {
      double d0 = 0.0;
      if (c.dm0 != 0.0) d0 = fma(0.5, rcp_grad(us), c.c) * (x * x) * c.dm0;
      phi[0] = in ? d0 : 0.0;
      phi[1] = in ? us : 0.0;
    }
  }
  // FP32 pass: u from (m0 - x)(m0 + x) and c u in FP64, the square root,
  // logarithm and reciprocal in single precision.
  struct C32 {
    double m0, im02, c, dm0;
  };
  __device__ static C32 load32(const double* ec) { return C32{ec[0], ec[1], ec[2], ec[3]}; }
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const double u64 = (c.m0 - x) * (c.m0 + x) * c.im02;
    const bool in = u64 > 0.0;
    const float us = in ? (float)u64 : 1.0f;
    const double cu = c.c * u64;
    const float xf = (float)x;
    if (LIN) {
      lam = in ? (float)cu : -__builtin_inff();
      gam = in ? xf * sqrt_f32(us) : 0.0f;
    } else {
      lam = in ? (float)fma(0.5, (double)log_f32(xf * xf * us), cu) : -__builtin_inff();
      gam = 1.0f;
    }
    if (GRAD) {
      float d0 = 0.0f;
      if (c.dm0 != 0.0) d0 = (float)(fma(0.5, (double)rcp_f32(us), c.c) * (x * x) * c.dm0);
      phi[0] = in ? d0 : 0.0f;
      phi[1] = in ? us : 0.0f;
    }
  }
};

// ------------------------------------------------------------------------
// Johnson S_U; linear (its factor 1/sqrt(1 + z^2) kept out of the log)
// ------------------------------------------------------------------------
// log g = -u^2/2 - ln sqrt(1 + z^2).  With s = sqrt(1 + z^2) and
// A = asinh z = sign(z) ln(|z| + s):
//   d log g/dmu     = w / lam,   w = u del / s + z / s^2
//   d log g/dlam    = w z / lam
//   d log g/dgam    = -u
//   d log g/ddel    = -u A
// Normalisation: u = gam + del asinh(z) maps g dx to (lam/del) e^{-u^2/2} du,
// so Z = (lam/del) sqrt(pi/2) [erf(u_hi/sqrt2) - erf(u_lo/sqrt2)]; dZ from
// the prefactor and the limits u_lo, u_hi.
struct JohnsonLeaf {
  static constexpr int kKind = kJohnson;
  static constexpr int NP = 4;
  static constexpr bool kLinear = true;
  static constexpr bool kEventLog = true;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  struct C {
    double mu, il, ga, de;
  };
  __device__ static bool valid(const double* p) { return p[1] > 0.0 && p[3] > 0.0; }
  __device__ static void consts(const double* p, LeafSetup& s) {
    const double il = 1.0 / p[1];
    s.ec[0] = p[0];
    s.ec[1] = il;
    s.ec[2] = p[2];
    s.ec[3] = p[3];
    s.fscale[0] = il;
    s.fscale[1] = il;
    s.fscale[2] = -1.0;
    s.fscale[3] = -1.0;
  }
  // the limits in u-space and what dZ needs of them
  struct Limits {
    double zl, zh, Al, Ah, ul, uh, sl, sh;
  };
  __device__ static Limits limits(const double* p, double lo, double hi) {
    Limits b;
    const double il = 1.0 / p[1];
    b.zl = (lo - p[0]) * il;
    b.zh = (hi - p[0]) * il;
    b.Al = asinh(b.zl);
    b.Ah = asinh(b.zh);
    b.ul = fma(p[3], b.Al, p[2]);
    b.uh = fma(p[3], b.Ah, p[2]);
    b.sl = sqrt(fma(b.zl, b.zl, 1.0));
    b.sh = sqrt(fma(b.zh, b.zh, 1.0));
    return b;
  }
  __device__ static void finish(const double* p, const Limits& b, double span, double el, double eh,
                                LeafSetup& s) {
    const double k = p[1] / p[3];
    s.Z = k * kSqrtPiOver2 * span;
    s.dZ[0] = el / b.sl - eh / b.sh;
    s.dZ[1] = s.Z / p[1] + b.zl * el / b.sl - b.zh * eh / b.sh;
    s.dZ[2] = k * (eh - el);
    s.dZ[3] = -s.Z / p[3] + k * (b.Ah * eh - b.Al * el);
  }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    consts(p, s);
    if (!analytic) return;
    const Limits b = limits(p, lo, hi);
    finish(p, b, erf_span(b.ul, b.uh), exp(-0.5 * b.ul * b.ul), exp(-0.5 * b.uh * b.uh), s);
  }
  // setup() over 4 lanes, as the Gaussian's: the two error-function values
  // and the two boundary exponentials each on a lane of their own (same
  // operations, same bits); complete on lane 0.
  static constexpr int kSetupLanes = 4;
  __device__ static void setup_coop(const double* p, double lo, double hi, bool analytic, LeafSetup& s, int lane) {
    consts(p, s);
    if (!analytic) return;
    const Limits b = limits(p, lo, hi);
    double v;
    if (lane >= 2) {
      const double t = lane == 2 ? b.ul : b.uh;
      v = exp(-0.5 * t * t);
    } else if (b.ul >= 0.0) {
      v = erfc((lane ? b.uh : b.ul) * kInvSqrt2);
    } else if (b.uh <= 0.0) {
      v = erfc((lane ? -b.ul : -b.uh) * kInvSqrt2);
    } else {
      v = erf((lane ? b.ul : b.uh) * kInvSqrt2);
    }
    const int base = (int)(threadIdx.x & 63) - lane;
    const double u0 = __shfl(v, base, 64), u1 = __shfl(v, base + 1, 64);
    const double el = __shfl(v, base + 2, 64), eh = __shfl(v, base + 3, 64);
    finish(p, b, u0 - u1, el, eh, s);
  }
  __device__ static double shape(const double* p, double, double, double x, double* dg) {
    const double z = (x - p[0]) / p[1];
    const double q = fma(z, z, 1.0), sq = sqrt(q);
    const double A = asinh(z);
    const double u = fma(p[3], A, p[2]);
    const double g = exp(-0.5 * u * u) / sq;
    const double w = u * p[3] / sq + z / q;
    dg[0] = g * w / p[1];
    dg[1] = g * w * z / p[1];
    dg[2] = -g * u;
    dg[3] = -g * u * A;
    return g;
  }
  __device__ static C load(const double* ec) { return C{ec[0], ec[1], ec[2], ec[3]}; }
  // LIN: lam = -u^2/2 and the linear factor 1/s; else the log of both.
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double z = (x - c.mu) * c.il;
    const double q = fma(z, z, 1.0);  // >= 1
    const double s = sqrt_pos(q);
    const double a = log_pos_tab(fabs(z) + s, g_log_tab);  // asinh |z|; the argument is >= 1
    const double A = copysign(a, z);
    const double u = fma(c.de, A, c.ga);
    const double r = rcp_full(s);
    if (LIN) {
      lam = -0.5 * u * u;
      gam = r;
    } else {
      lam = fma(-0.5, log_pos_tab(q, g_log_tab), -0.5 * u * u);
      gam = 1.0;
    }
    if (GRAD) {
      const double w = fma(u * c.de, r, z * (r * r));
      phi[0] = w;
      phi[1] = w * z;
      phi[2] = u;
      phi[3] = u * A;
    }
  }
  // FP32 pass: x - mu in FP64, z, the square root, logarithm and reciprocal
  // in single precision; u = gam + del A (a per-point constant added) and
  // u^2 in FP64.
  struct C32 {
    double mu, ga, de;
    F2 il;
  };
  __device__ static C32 load32(const double* ec) { return C32{ec[0], ec[2], ec[3], split2(ec[1])}; }
  template <bool GRAD, bool LIN = false>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float z = mul2((float)(x - c.mu), c.il);
    const float q = fmaf(z, z, 1.0f);
    const float s = sqrt_f32(q);
    const float A = copysignf(log_f32(fabsf(z) + s), z);
    const double u64 = fma(c.de, (double)A, c.ga);
    const float r = rcp_f32(s);
    if (LIN) {
      lam = (float)(-0.5 * u64 * u64);
      gam = r;
    } else {
      lam = (float)fma(-0.5, (double)log_f32(q), -0.5 * u64 * u64);
      gam = 1.0f;
    }
    if (GRAD) {
      const float u = (float)u64;
      const float w = fmaf((float)(u64 * c.de), r, z * (r * r));
      phi[0] = w;
      phi[1] = w * z;
      phi[2] = u;
      phi[3] = u * A;
    }
  }
};

// ------------------------------------------------------------------------
// Chi-square with nu degrees of freedom
// ------------------------------------------------------------------------
// log g = (nu/2 - 1) ln x - x/2, d log g/dnu = ln(x)/2: one logarithm per
// event.  Z over [lo, hi] (0 <= lo, hi <= 1000) = 2^k [gamma(k, hi/2) -
// gamma(k, lo/2)] with k = nu/2 and the lower incomplete gamma function
//   gamma(k, y) = y^k e^{-y} sum_n t_n,  t_n = y^n / (k (k+1) ... (k+n)),
// whose k-derivative is gamma ln y - y^k e^{-y} sum_n t_n H_n with
// H_n = sum_{j<=n} 1/(k+j); the terms are positive, so the partial sums
// have no cancellation.  About y + 10 sqrt(y) + 20 terms, on one lane in the
// per-point prologue: each term costs one refined reciprocal (no division),
// and the stopping test is taken every 4 terms.
__device__ inline void lower_gamma_dk(double k, double y, double& g, double& dg) {
  g = 0.0;
  dg = 0.0;
  if (!(y > 0.0)) return;
  double kn = k;
  double h = rcp_full(kn);
  double S = 0.0, D = 0.0, t = h, H = h;
  for (int n = 0; n < 4096; n += 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      S += t;
      D = fma(t, H, D);
      kn += 1.0;
      h = rcp_full(kn);
      t *= y * h;
      H += h;
    }
    if (n + 3 > y && t < 1e-18 * S) break;
  }
  const double ly = log(y);
  const double pre = exp(fma(k, ly, -y));
  g = pre * S;
  dg = fma(g, ly, -pre * D);
}

struct Chi2Leaf {
  static constexpr int kKind = kChi2;
  static constexpr int NP = 1;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = true;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = false;       // no per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised by the shared rules (closed form or one GL rule)
  struct C {
    double km1;  // nu/2 - 1
  };
  __device__ static bool valid(const double* p) { return p[0] > 0.0; }
  __device__ static void consts(const double* p, LeafSetup& s) {
    s.ec[0] = fma(0.5, p[0], -1.0);
    s.fscale[0] = 0.5;
  }
  __device__ static void finish(double k, double ga, double dga, double gb, double dgb, LeafSetup& s) {
    const double p2 = exp2(k);
    s.Z = p2 * (gb - ga);
    s.dZ[0] = 0.5 * fma(kLn2, s.Z, p2 * (dgb - dga));
  }
  __device__ static void setup(const double* p, double lo, double hi, bool analytic, LeafSetup& s) {
    consts(p, s);
    if (!analytic) return;
    const double k = 0.5 * p[0];
    double ga, dga, gb, dgb;
    lower_gamma_dk(k, 0.5 * lo, ga, dga);
    lower_gamma_dk(k, 0.5 * hi, gb, dgb);
    finish(k, ga, dga, gb, dgb, s);
  }
  // setup() over 2 lanes: the series at hi on lane 0, at lo on lane 1.
  static constexpr int kSetupLanes = 2;
  __device__ static void setup_coop(const double* p, double lo, double hi, bool analytic, LeafSetup& s, int lane) {
    consts(p, s);
    if (!analytic) return;
    const double k = 0.5 * p[0];
    double g, dg;
    lower_gamma_dk(k, 0.5 * (lane ? lo : hi), g, dg);
    const int base = (int)(threadIdx.x & 63) - lane;
    const double gb = __shfl(g, base, 64), dgb = __shfl(dg, base, 64);
    const double ga = __shfl(g, base + 1, 64), dga = __shfl(dg, base + 1, 64);
    finish(k, ga, dga, gb, dgb, s);
  }
  __device__ static double shape(const double* p, double, double, double x, double* dg) {
    const double lx = log(x);
    const double g = exp(fma(fma(0.5, p[0], -1.0), lx, -0.5 * x));
    dg[0] = 0.5 * g * lx;
    return g;
  }
  // the integrand on [0, hi] after x = s^2 (dx = 2 s ds): 2 s^{nu-1} e^{-s^2/2}
  __device__ static double shape_subst(const double* p, double sv, double* dg) {
    const double ls = log(sv);
    const double g = 2.0 * exp(fma(p[0] - 1.0, ls, -0.5 * sv * sv));
    dg[0] = g * ls;
    return g;
  }
  __device__ static C load(const double* ec) { return C{ec[0]}; }
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double lx = x > 0.0 ? log_pos_tab(x, g_log_tab) : -__builtin_inf();  // x = 0: p = 0 or inf (flagged)
    lam = fma(c.km1, lx, -0.5 * x);
    gam = 1.0;
    if (GRAD) phi[0] = lx;
  }
  // FP32 pass: the logarithm in single precision, corrected to first order
  // for the rounding of x to single; the combination in FP64.
  struct C32 {
    double km1;
  };
  __device__ static C32 load32(const double* ec) { return C32{ec[0]}; }
  template <bool GRAD>
  __device__ static inline void event32(double x, const C32& c, float& lam, float& gam, float* phi) {
    const float xf = (float)x;
    double lx = -__builtin_inf();
    if (x > 0.0) lx = (double)log_f32(xf) + (x - (double)xf) * (double)rcp_f32(xf);
    lam = (float)fma(c.km1, lx, -0.5 * x);
    gam = 1.0f;
    if (GRAD) phi[0] = (float)lx;
  }
};

static_assert(sizeof(PerTheta::ec[0]) == sizeof(LeafSetup::ec), "leaf constant rows must match");
// every leaf's constants fit one row: CB uses 11, Chebyshev 2 + K (K <= 8)
static_assert(11 <= kLeafConsts && 2 + 8 <= kLeafConsts, "leaf constants");

}  // namespace nllmi

#include "hypatia.h"
#include "jit_leaf.h"
