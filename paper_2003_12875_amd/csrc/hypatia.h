// hypatia.h -- the Hypatia2 leaf on the device: the two-sided Hypatia
// density (a generalised hyperbolic core of width sigma continued on both
// sides by power laws, Santos and Dupertuis 2014), one of the densities the
// paper's Sec. 3 adds to RooFit's built-in ones.
//
// Parameters (mu, sigma, lambda, zeta, beta, a_l, n_l, a_r, n_r); with
// d = x - mu, nu = lambda - 1/2, A^2 = zeta K_lambda(zeta)/K_{lambda+1}(zeta),
// delta^2 = A^2 sigma^2, alpha = zeta/delta, r^2 = d^2 + delta^2, z = alpha r:
//   core  log g = (nu/2) ln r^2 + beta d + ln K_nu(z)   for d_l <= d <= d_h,
//   low   log g = log G_l - n_l ln(1 + k_l (d_l - d))  for d < d_l = -a_l sigma,
//   high  log g = log G_h - n_r ln(1 + k_h (d - d_h))  for d > d_h = a_r sigma,
// G_l, G_h the core's values at the junctions, k_l = s_l/n_l and
// k_h = -s_h/n_r from the core's log-slopes there (s_l > 0 > s_h), so the
// tails continue the core with equal value and slope.
//
// K_nu has no closed form, so per parameter point the block computes (all
// threads, with barriers) tables of three smooth functions of s = ln z on
// the core's z-range -- ln K_nu(z) + z, (K_{nu+1}(z)/K_nu(z) - 1) z and
// d ln K_nu(z)/d nu -- as Chebyshev interpolants of degree 15 on up to 8
// panels of width <= 1.2 in s, from K values by the trapezoidal rule on
// K_nu(z) e^z = int_0^inf e^{-z (cosh t - 1)} cosh(nu t) dt (step
// min(1/4, 0.45 (z^2 + (|nu|+1)^2)^(-1/4)), converged to ~1e-14 relative
// for |nu| <= 6, 1e-3 <= z <= 700 against 30-digit values).  The per-event
// pass then evaluates the core by one table logarithm, one square root and
// three Clenshaw sums.  Derivatives: the core's by the chain through
// (d, delta^2, alpha, nu, beta), with Q = K_{nu+1}/K_nu and
// K_nu'/K_nu = nu/z - Q; the junction quantities' (for the tails) with the
// second derivatives Q' = Q^2 - (2 nu + 1) Q/z - 1 and
// d Q/d nu = Q (d ln K_{nu+1}/d nu - d ln K_nu/d nu), evaluated exactly at
// the two junctions.  Normalisation: 256-point Gauss-Legendre on the core
// in u = asinh(d/delta) (smooth in u however narrow the peak) and on each
// tail in v = ln(1 + k w) (a power law becomes an exponential).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "fp64.h"
#include "plan.h"

namespace nllmi {

// scalar slots of the per-point table (after the interpolant coefficients)
enum HypSlot : int {
  hMu, hDelta2, hAlpha, hLnAlpha, hNu, hBeta, hDl, hDh, hS0, hInvW, hNPan, hRef,
  hCsd, hCsa, hCld, hCla, hCzd, hCza, hLGl, hKl, hNl, hLGh, hKh, hNr, hLamFree,
  hDelta, hOk, hInvAlpha, hNuOverAlpha, hBadJ, hNumSlots
};
static_assert(hNumSlots <= 32, "Hypatia2 scalar slots");
constexpr int kHypFn = kHypPanels * kHypDeg;  // coefficients of one function

// broadcast lane 0's value (kept in scalar registers)
__device__ inline double uniform_d(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// K_nu(z) e^z, K_{nu+1}(z) e^z and their derivatives in the order, as four
// trapezoidal sums over t (see the header); z > 0.  A group of G
// consecutive lanes of one wave (G a power of 2, the group aligned to G)
// computes one set of sums: lane r takes the terms j = r, r + G, ... in
// rounds of G terms; each round's terms are added across the group (xor
// butterfly) to sums that every lane of the group holds, and the sums stop
// after the first round whose every term is negligible against them (past
// the integrand's peak, t > 1 and z sinh t above the orders).  The order
// of the additions depends on G only.
__device__ inline void bessel_k4(double nu, double z, double out[4], int G, int r) {
  const double a0 = fabs(nu), a1 = fabs(nu + 1.0);
  const double g0 = nu < 0.0 ? -1.0 : 1.0, g1 = nu + 1.0 < 0.0 ? -1.0 : 1.0;
  const double h = fmin(0.25, 0.45 / sqrt(sqrt(z * z + (a0 + 1.0) * (a0 + 1.0))));
  const double mono = fmax(a0, a1) + 1.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int base = 0; base < 8192; base += G) {
    const int j = base + r;
    const double t = j * h;
    const double et = exp(t);
    const double ch = 0.5 * (et + 1.0 / et), sh = 0.5 * (et - 1.0 / et);
    const double E = exp(-z * (ch - 1.0));
    const double m0 = expm1(a0 * t), p0 = 1.0 + m0;
    const double m1 = expm1(a1 * t), p1 = 1.0 + m1;
    double c0 = 0.5 * (p0 + 1.0 / p0), d0 = g0 * 0.5 * m0 * (1.0 + 1.0 / p0);
    double c1 = 0.5 * (p1 + 1.0 / p1), d1 = g1 * 0.5 * m1 * (1.0 + 1.0 / p1);
    const double w = j == 0 ? 0.5 * E : E;
    const double u0 = w * c0, u1 = w * c1, u2 = w * t * d0, u3 = w * t * d1;
    double v0 = u0, v1 = u1, v2 = u2, v3 = u3;
    for (int off = 1; off < G; off <<= 1) {
      v0 += __shfl_xor(v0, off, 64);
      v1 += __shfl_xor(v1, off, 64);
      v2 += __shfl_xor(v2, off, 64);
      v3 += __shfl_xor(v3, off, 64);
    }
    s0 += v0;
    s1 += v1;
    s2 += v2;
    s3 += v3;
    int done = t > 1.0 && z * sh > mono && u0 <= 1e-18 * s0 && u1 <= 1e-18 * s1 &&
               fabs(u2) <= 1e-18 * fabs(s2) + 1e-300 && fabs(u3) <= 1e-18 * fabs(s3) + 1e-300;
    for (int off = 1; off < G; off <<= 1) done &= __shfl_xor(done, off, 64);
    if (done) break;
  }
  out[0] = h * s0;
  out[1] = h * s1;
  out[2] = h * s2;
  out[3] = h * s3;
}

// sum_k c[k] T_k(y), k < kHypDeg (c[0] already halved)
__device__ __forceinline__ double hyp_clenshaw(const double* __restrict__ c, double y) {
  const double y2 = y + y;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kHypDeg - 1; k >= 1; --k) {
    const double b0 = fma(y2, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(y, b1, c[0] - b2);
}

struct HypatiaLeaf {
  static constexpr int kKind = kHypatia;
  static constexpr int NP = 9;
  static constexpr bool kLinear = false;
  static constexpr bool kEventLog = true;  // a logarithm per event (FP64 pass)
  static constexpr bool kAux = true;       // per-point tables beside PerTheta
  static constexpr bool kOwnNorm = false;   // normalised through gl_norm on its tables
  static constexpr int kSetupLanes = 1;

  __device__ static bool valid(const double* p) {
    return p[1] > 0.0 && p[3] > 0.0 && p[5] > 0.0 && p[6] > 1.0 && p[7] > 0.0 && p[8] > 1.0;
  }

  struct C32 {};  // no FP32-compensated pass for this leaf
  // the per-event constants (uniform: scalar registers) and the table
  struct C {
    const double* aux;  // interpolant coefficients and tail tables
    double mu, delta2, dl, dh, ref, lnalpha, s0, invw, alpha, invalpha, nu, beta, nuoa;
    double csd, csa, cld, cla, czd, cza, kl, kh, nl, nr, lgl, lgh;
    int npan, lamfree;
  };
  __device__ static C load_aux(const double* aux) {
    const double* sc = aux + kHypScal;
    C c;
    c.aux = aux;
    c.mu = uniform_d(sc[hMu]);
    c.delta2 = uniform_d(sc[hDelta2]);
    c.dl = uniform_d(sc[hDl]);
    c.dh = uniform_d(sc[hDh]);
    c.ref = uniform_d(sc[hRef]);
    c.lnalpha = uniform_d(sc[hLnAlpha]);
    c.s0 = uniform_d(sc[hS0]);
    c.invw = uniform_d(sc[hInvW]);
    c.alpha = uniform_d(sc[hAlpha]);
    c.invalpha = uniform_d(sc[hInvAlpha]);
    c.nu = uniform_d(sc[hNu]);
    c.beta = uniform_d(sc[hBeta]);
    c.nuoa = uniform_d(sc[hNuOverAlpha]);
    c.csd = uniform_d(sc[hCsd]);
    c.csa = uniform_d(sc[hCsa]);
    c.cld = uniform_d(sc[hCld]);
    c.cla = uniform_d(sc[hCla]);
    c.czd = uniform_d(sc[hCzd]);
    c.cza = uniform_d(sc[hCza]);
    c.kl = uniform_d(sc[hKl]);
    c.kh = uniform_d(sc[hKh]);
    c.nl = uniform_d(sc[hNl]);
    c.nr = uniform_d(sc[hNr]);
    c.lgl = uniform_d(sc[hLGl]);
    c.lgh = uniform_d(sc[hLGh]);
    c.npan = (int)uniform_d(sc[hNPan]);
    c.lamfree = uniform_d(sc[hLamFree]) != 0.0 ? 1 : 0;
    return c;
  }

  // core log-density (without the reference) and its features at d (F:
  // d/dd, d/d delta^2, d/d alpha, d/d nu, d/d beta of it); the logarithm of
  // r^2 and r given
  template <bool GRAD>
  __device__ static inline double core(const C& c, double d, double lr2, double r, double* F) {
    const double s = fma(0.5, lr2, c.lnalpha);
    const double tt = (s - c.s0) * c.invw;
    int pn = (int)tt;
    pn = pn < 0 ? 0 : (pn >= c.npan ? c.npan - 1 : pn);
    // clamped: tail events evaluate the core too (and discard it)
    const double y = fmin(fmax(fma(2.0, tt - (double)pn, -1.0), -1.0), 1.0);
    const double* cf = c.aux + pn * kHypDeg;
    const double z = c.alpha * r;
    const double g1 = hyp_clenshaw(cf, y);
    const double L = fma(0.5 * c.nu, lr2, fma(c.beta, d, g1 - z));
    if constexpr (GRAD) {
      const double h2 = hyp_clenshaw(cf + kHypFn, y);
      const double f3 = c.lamfree ? hyp_clenshaw(cf + 2 * kHypFn, y) : 0.0;
      const double ir = rcp_grad(r);
      const double Q = fma(h2, ir * c.invalpha, 1.0);
      const double ir2 = ir * ir;
      F[0] = fma(2.0 * c.nu * d, ir2, c.beta) - c.alpha * d * ir * Q;
      F[1] = fma(c.nu, ir2, -0.5 * c.alpha * Q * ir);
      F[2] = c.nuoa - r * Q;
      F[3] = fma(0.5, lr2, f3);
      F[4] = d;
    }
    return L;
  }

  // -------- per parameter point (all threads of the block) --------------
  template <int NT>
  __device__ static void setup_aux(const double* p, double lo, double hi, double* aux) {
    static_assert(NT >= 256 && kHypPanels * kHypDeg <= 192, "node lanes below the junction lanes 192..255");
    double* sc = aux + kHypScal;
    double* tl = aux + kHypTails;  // [2][9][3]
    const int t = threadIdx.x;
    const bool ok0 = valid(p);
    // A^2 from K_lambda(zeta), K_{lambda+1}(zeta): the sums over wave 0's
    // 64 lanes, the rest on lane 0
    double S0[4];
    if (t < 64 && ok0) bessel_k4(p[2], p[3], S0, 64, t);
    if (t == 0) {
      sc[hOk] = ok0 ? 1.0 : 0.0;
      sc[hBadJ] = 0.0;  // set by the junction lanes (hOk is read before they run)
      if (ok0) {
        const double sg = p[1], la = p[2], ze = p[3];
        const double* S = S0;
        const double A2 = ze * S[0] / S[1];
        const double Ql = S[1] / S[0];
        const double dl2 = S[2] / S[0] - S[3] / S[1];                 // d ln A^2 / d lambda
        const double dz2 = (2.0 * la + 2.0) / ze - Ql + 1.0 / Ql;      // d ln A^2 / d zeta
        const double delta2 = A2 * sg * sg, delta = sqrt(delta2), alpha = ze / delta;
        const double nu = la - 0.5;
        sc[hMu] = p[0];
        sc[hDelta2] = delta2;
        sc[hDelta] = delta;
        sc[hAlpha] = alpha;
        sc[hInvAlpha] = 1.0 / alpha;
        sc[hLnAlpha] = log(alpha);
        sc[hNu] = nu;
        sc[hNuOverAlpha] = nu / alpha;
        sc[hBeta] = p[4];
        sc[hCsd] = 2.0 * sg * A2;
        sc[hCsa] = -alpha / sg;
        sc[hCld] = delta2 * dl2;
        sc[hCla] = -0.5 * alpha * dl2;
        sc[hCzd] = delta2 * dz2;
        sc[hCza] = alpha / ze - 0.5 * alpha * dz2;
        const double dl = -p[5] * sg, dh = p[7] * sg, dm = fmax(-dl, dh);
        sc[hDl] = dl;
        sc[hDh] = dh;
        sc[hNl] = p[6];
        sc[hNr] = p[8];
        const double s0 = log(ze), s1 = log(alpha * sqrt(fma(dm, dm, delta2)));
        const double W = s1 - s0;
        const double np = fmax(1.0, ceil(W / 1.2));
        sc[hS0] = s0;
        sc[hNPan] = fmin(np, (double)kHypPanels);
        sc[hInvW] = sc[hNPan] / W;
        sc[hLamFree] = 1.0;
        if (!(np <= (double)kHypPanels) || !__builtin_isfinite(W) || !(W > 0.0)) sc[hOk] = 0.0;
      }
    }
    __syncthreads();
    if (sc[hOk] == 0.0) return;  // uniform
    const double nu = sc[hNu], delta2 = sc[hDelta2], alpha = sc[hAlpha], beta = sc[hBeta];
    const int npan = (int)sc[hNPan];
    // interpolation nodes on lanes 0..191: node n = npan * kHypDeg at most
    // (panel n / kHypDeg) on the G lanes [n G, n G + G), G the largest power
    // of 2 (at most 64) with npan * kHypDeg * G <= 192; its lane 0 keeps it
    const int n_nodes = npan * kHypDeg;
    int G = 64;
    while (G > 1 && n_nodes * G > 192) G >>= 1;
    double nv[3] = {0.0, 0.0, 0.0};
    const int nd = t / G, nr = t % G;
    const bool node = t < 192 && nd < n_nodes;
    if (node) {
      const int pn = nd / kHypDeg, jj = nd % kHypDeg;
      const double y = cospi(((double)jj + 0.5) / kHypDeg);
      const double s = sc[hS0] + ((double)pn + 0.5 * (y + 1.0)) / sc[hInvW];
      const double z = exp(s);
      double S[4];
      bessel_k4(nu, z, S, G, nr);
      nv[0] = log(S[0]);
      nv[1] = (S[1] / S[0] - 1.0) * z;
      nv[2] = S[2] / S[0];
    }
    // junctions, beside the nodes: lanes 192..223 the low one, 224..255 the
    // high one (32 lanes each for the sums, the rest on the first)
    if (t >= 192 && t < 256) {
      const bool low = t < 224;
      const double d = low ? sc[hDl] : sc[hDh];
      const double r2 = fma(d, d, delta2), r = sqrt(r2), z = alpha * r;
      double S[4];
      bessel_k4(nu, z, S, 32, t & 31);
      if ((t & 31) == 0) {
        const double lr2 = log(r2);
        const double lk = log(S[0]) - z;
        const double Q = S[1] / S[0], f3 = S[2] / S[0], f4 = S[3] / S[1];
        const double L = fma(0.5 * nu, lr2, fma(beta, d, lk));
        const double Fd = 2.0 * nu * d / r2 + beta - alpha * d / r * Q;
        const double Fdl = nu / r2 - 0.5 * alpha * Q / r;
        const double Fal = nu / alpha - r * Q;
        const double Fnu = 0.5 * lr2 + f3;
        const double Qp = Q * Q - (2.0 * nu + 1.0) * Q / z - 1.0;
        const double dQnu = Q * (f4 - f3);
        const double r3 = r2 * r;
        const double Gdd = 2.0 * nu * (r2 - 2.0 * d * d) / (r2 * r2) - alpha * delta2 * Q / r3 -
                           alpha * alpha * d * d * Qp / r2;
        const double Gdl = -2.0 * nu * d / (r2 * r2) + alpha * d * Q / (2.0 * r3) - alpha * alpha * d * Qp / (2.0 * r2);
        const double Gal = -(d / r) * (Q + z * Qp);
        const double Gnu = 2.0 * d / r2 - alpha * d / r * dQnu;
        const double n = low ? sc[hNl] : sc[hNr];
        const double sl = Fd;  // the log-slope at the junction
        const double k = low ? sl / n : -sl / n;
        const int nidx = low ? 6 : 8;
        if (low) {
          sc[hLGl] = L;
          sc[hKl] = k;
          sc[hRef] = L;
        } else {
          sc[hLGh] = L;
          sc[hKh] = k;
        }
        if (!(k > 0.0) || !__builtin_isfinite(L)) sc[hBadJ] = 1.0;
        double* tab = tl + (low ? 0 : 27);
        for (int q = 0; q < NP; ++q) {
          const double dd = q == 1 ? (low ? -p[5] : p[7]) : (q == 5 && low ? -p[1] : (q == 7 && !low ? p[1] : 0.0));
          const double ddl = q == 1 ? sc[hCsd] : (q == 2 ? sc[hCld] : (q == 3 ? sc[hCzd] : 0.0));
          const double dal = q == 1 ? sc[hCsa] : (q == 2 ? sc[hCla] : (q == 3 ? sc[hCza] : 0.0));
          const double dnu = q == 2 ? 1.0 : 0.0, dbe = q == 4 ? 1.0 : 0.0;
          const double dL = Fd * dd + Fdl * ddl + Fal * dal + Fnu * dnu + d * dbe;
          const double ds = Gdd * dd + Gdl * ddl + Gal * dal + Gnu * dnu + dbe;
          const double dk = (low ? ds : -ds) / n - (q == nidx ? k / n : 0.0);
          const double dw = low ? dd + (q == 0 ? 1.0 : 0.0) : -dd - (q == 0 ? 1.0 : 0.0);
          tab[3 * q] = dL;
          tab[3 * q + 1] = n * dk;
          tab[3 * q + 2] = n * k * dw;
        }
      }
    }
    // node values into the coefficient area, then the coefficients
    if (node && nr == 0) {
      const int pn = nd / kHypDeg, jj = nd % kHypDeg;
      for (int f = 0; f < 3; ++f) aux[f * kHypFn + pn * kHypDeg + jj] = nv[f];
    }
    __syncthreads();
    // coefficients c_k = (2 / N) sum_j v_j cos(pi k (j + 1/2) / N) (c_0
    // halved), computed from the node values and written over them
    constexpr int kPer = (kHypCoef + NT - 1) / NT;
    const int ncoef = 3 * npan * kHypDeg;
    double cval[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = t + e * NT;
      cval[e] = 0.0;
      if (i < ncoef) {
        const int f = i / (npan * kHypDeg), rest = i % (npan * kHypDeg), pn = rest / kHypDeg, k = rest % kHypDeg;
        const double* v = aux + f * kHypFn + pn * kHypDeg;
        double acc = 0.0;
        for (int jj = 0; jj < kHypDeg; ++jj) acc = fma(v[jj], cospi((double)k * ((double)jj + 0.5) / kHypDeg), acc);
        cval[e] = acc * ((k == 0 ? 1.0 : 2.0) / kHypDeg);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = t + e * NT;
      if (i < ncoef) aux[(i / (npan * kHypDeg)) * kHypFn + i % (npan * kHypDeg)] = cval[e];
    }
    __syncthreads();
  }

  // the tables describe a valid density (uniform)
  __device__ static bool aux_ok(const double* aux) {
    return aux[kHypScal + hOk] != 0.0 && aux[kHypScal + hBadJ] == 0.0;
  }

  // one thread's Gauss-Legendre contributions to Z and dZ (v[0], v[1..9]):
  // node i of the core in u = asinh(d/delta) and of each tail in
  // v = ln(1 + k w); the values relative to exp(ref) (ref: the left
  // junction's log value), features as the event pass forms them
  __device__ static void gl_norm(const double* aux, double lo, double hi, const double* glx, const double* glw,
                                 double (&v)[NP + 1]) {
    const double* sc = aux + kHypScal;
    const double* tl = aux + kHypTails;
#pragma unroll
    for (int j = 0; j <= NP; ++j) v[j] = 0.0;
    if (!aux_ok(aux)) {
      v[0] = __builtin_nan("");
      return;
    }
    const int i = threadIdx.x;
    const double mu = sc[hMu], dl = sc[hDl], dh = sc[hDh], delta = sc[hDelta], ref = sc[hRef];
    const double a = lo - mu, b = hi - mu;
    // core
    const double ca = fmax(a, dl), cb = fmin(b, dh);
    if (cb > ca) {
      const double ua = asinh(ca / delta), ub = asinh(cb / delta);
      const double hw = 0.5 * (ub - ua), u = fma(hw, glx[i], 0.5 * (ua + ub));
      const double d = delta * sinh(u), r = delta * cosh(u);
      const double lr2 = 2.0 * log(r);
      double F[5];
      const double L = core<true>(load_aux(aux), d, lr2, r, F);
      const double g = exp(L - ref) * hw * glw[i] * r;
      v[0] += g;
      v[1] += g * -F[0];
      v[2] += g * fma(sc[hCsd], F[1], sc[hCsa] * F[2]);
      v[3] += g * (F[3] + fma(sc[hCld], F[1], sc[hCla] * F[2]));
      v[4] += g * fma(sc[hCzd], F[1], sc[hCza] * F[2]);
      v[5] += g * d;
    }
    // tails: w from the junction, D = 1 + k w = e^v
    for (int side = 0; side < 2; ++side) {
      const bool low = side == 0;
      const double wa = low ? fmax(0.0, dl - b) : fmax(0.0, a - dh);
      const double wb = low ? dl - a : b - dh;
      if (!(wb > wa)) continue;
      const double k = low ? sc[hKl] : sc[hKh], n = low ? sc[hNl] : sc[hNr];
      const double lG = low ? sc[hLGl] : sc[hLGh];
      const double* tab = tl + (low ? 0 : 27);
      const int nidx = low ? 6 : 8;
      const double va = log1p(k * wa), vb = log1p(k * wb);
      const double hw = 0.5 * (vb - va), vv = fma(hw, glx[i], 0.5 * (va + vb));
      const double D = exp(vv), w = expm1(vv) / k, iD = 1.0 / D;
      const double g = exp(fma(-n, vv, lG) - ref) * hw * glw[i] * D / k;
      v[0] += g;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const double ph = tab[3 * q] - (q == nidx ? vv : 0.0) - tab[3 * q + 1] * w * iD - tab[3 * q + 2] * iD;
        v[1 + q] += g * ph;
      }
    }
  }

  // -------- the event pass -----------------------------------------------
  template <bool GRAD>
  __device__ static inline void event(double x, const C& c, double& lam, double& gam, double* phi) {
    const double d = x - c.mu;
    const double r2 = fma(d, d, c.delta2);
    const double lr2 = log_pos_tab(r2, g_log_tab);
    const double r = sqrt_pos(r2);
    double F[5];
    double L = core<GRAD>(c, d, lr2, r, F);
    if constexpr (GRAD) {
      phi[0] = -F[0];
      phi[1] = fma(c.csd, F[1], c.csa * F[2]);
      phi[2] = F[3] + fma(c.cld, F[1], c.cla * F[2]);
      phi[3] = fma(c.czd, F[1], c.cza * F[2]);
      phi[4] = d;
#pragma unroll
      for (int q = 5; q < NP; ++q) phi[q] = 0.0;
    }
    const bool lo_t = d < c.dl, hi_t = d > c.dh;
    if (lo_t || hi_t) {  // the power-law tails (a real branch: few events)
      const double w = lo_t ? c.dl - d : d - c.dh;
      const double k = lo_t ? c.kl : c.kh, n = lo_t ? c.nl : c.nr;
      const double lG = lo_t ? c.lgl : c.lgh;
      const double D = fma(k, w, 1.0);
      const double lD = log_pos_tab(D, g_log_tab);
      L = fma(-n, lD, lG);
      if constexpr (GRAD) {
        const double* tab = c.aux + kHypTails + (lo_t ? 0 : 27);
        const int nidx = lo_t ? 6 : 8;
        const double iD = rcp_grad(D), wD = w * iD;
#pragma unroll
        for (int q = 0; q < NP; ++q)
          phi[q] = tab[3 * q] - (q == nidx ? lD : 0.0) - tab[3 * q + 1] * wD - tab[3 * q + 2] * iD;
      }
    }
    lam = L - c.ref;
    gam = 1.0;
  }
};

}  // namespace nllmi
