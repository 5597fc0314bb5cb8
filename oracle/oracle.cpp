/*
 * oracle.cpp -- scalar FP64 reference evaluator (test infrastructure only;
 * the product path never links it).  See oracle.h for the contract.
 *
 * Everything here is written to be checked by eye against the paper and
 * the textbook definitions of the densities:
 *   - the likelihood is evaluated event by event, the classic single-value
 *     way of Sec. 5.1: values are written into the leaves, the top node's
 *     probability is obtained recursively from its daughters and their
 *     normalisation, and parameter-only quantities (normalisation
 *     integrals) are computed once per parameter point;
 *   - densities are composed in the linear domain, p = sum c_j p_j for a
 *     sum and p = prod p_d for a product, exactly as defined;
 *   - derivatives are propagated forward through the same recursion;
 *   - every sum over events is Neumaier-compensated FP64.
 * Valid while every p(x_i) is a normal double (no underflow to 0).
 */
#include "oracle.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
constexpr double kPi = 3.141592653589793238462643383279502884;

/* Neumaier's improvement of Kahan summation. */
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double v) {
    double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule: roots of P_n by Newton's method on the three-   */
/* term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, carried in */
/* long double; weights w = 2 / ((1 - x^2) P_n'(x)^2).                  */
/* ------------------------------------------------------------------ */
struct Rule {
  std::vector<double> x, w;
};

Rule make_rule(int n) {
  Rule r;
  r.x.assign(n, 0.0);
  r.w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0.0L;
    for (int it = 0; it < 200; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int k = 1; k < n; ++k) {
        long double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      long double step = p1 / dp;
      z -= step;
      if (fabsl(step) < 1e-21L) break;
    }
    {
      long double p0 = 1.0L, p1 = z;
      for (int k = 1; k < n; ++k) {
        long double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
    }
    long double wt = 2.0L / ((1.0L - z * z) * dp * dp);
    r.x[n - 1 - i] = (double)z;
    r.x[i] = (double)(-z);
    r.w[n - 1 - i] = (double)wt;
    r.w[i] = (double)wt;
  }
  if (n % 2 == 1) r.x[n / 2] = 0.0;
  return r;
}

const Rule& rule256() {
  static const Rule r = make_rule(256);
  return r;
}

/* ------------------------------------------------------------------ */
/* Unnormalised leaf shapes g(x; theta) and dg/dtheta_local.            */
/* ------------------------------------------------------------------ */
inline double P(const double* th, const orc_node& nd, int k) { return th[nd.param[k]]; }

/* Gaussian: g = exp(-t^2/2), t = (x - mu)/sigma. */
double g_gauss(const orc_node& nd, const double* th, double x, double* dg) {
  double mu = P(th, nd, 0), s = P(th, nd, 1);
  double t = (x - mu) / s;
  double g = std::exp(-0.5 * t * t);
  if (dg) {
    dg[0] = g * t / s;
    dg[1] = g * t * t / s;
  }
  return g;
}

/* Exponential: g = exp(c x). */
double g_exp(const orc_node& nd, const double* th, double x, double* dg) {
  double c = P(th, nd, 0);
  double g = std::exp(c * x);
  if (dg) dg[0] = g * x;
  return g;
}

/* Chebyshev series of the first kind on [lo, hi] with the T_0 coefficient
 * fixed at 1: g = 1 + sum_{k=1..K} a_k T_k(x'), x' = (2x - lo - hi)/(hi - lo). */
double g_cheb(const orc_node& nd, const double* th, double lo, double hi, double x,
              double* dg) {
  double y = (2.0 * x - lo - hi) / (hi - lo);
  double tkm1 = 1.0, tk = y, g = 1.0;
  for (int k = 1; k <= nd.n_param; ++k) {
    g += P(th, nd, k - 1) * tk;
    if (dg) dg[k - 1] = tk;
    double tkp1 = 2.0 * y * tk - tkm1;
    tkm1 = tk;
    tk = tkp1;
  }
  return g;
}

/* Crystal Ball with a power-law tail on the low side:
 *   t > -alpha : exp(-t^2/2)
 *   t <= -alpha: A (B - t)^(-n),  A = (n/alpha)^n exp(-alpha^2/2),
 *                                 B = n/alpha - alpha.                  */
double g_cb(const orc_node& nd, const double* th, double x, double* dg) {
  double m0 = P(th, nd, 0), s = P(th, nd, 1), a = P(th, nd, 2), n = P(th, nd, 3);
  double t = (x - m0) / s;
  if (t > -a) {
    double g = std::exp(-0.5 * t * t);
    if (dg) {
      dg[0] = g * t / s;
      dg[1] = g * t * t / s;
      dg[2] = 0.0;
      dg[3] = 0.0;
    }
    return g;
  }
  double A = std::pow(n / a, n) * std::exp(-0.5 * a * a);
  double B = n / a - a;
  double D = B - t;
  double g = A * std::pow(D, -n);
  if (dg) {
    dg[0] = g * (-n / (s * D));
    dg[1] = g * (-n * t / (s * D));
    dg[2] = g * (-n / a - a + n * (n / (a * a) + 1.0) / D);
    dg[3] = g * (std::log(n / a) + 1.0 - std::log(D) - n / (a * D));
  }
  return g;
}

/* ARGUS with power 1/2: g = m sqrt(u) exp(c u), u = 1 - (m/m0)^2, for
 * m < m0, and 0 otherwise.  u is formed as (m0 - m)(m0 + m)/m0^2.       */
double g_argus(const orc_node& nd, const double* th, double x, double* dg) {
  double m0 = P(th, nd, 0), c = P(th, nd, 1);
  if (x >= m0) {
    if (dg) dg[0] = dg[1] = 0.0;
    return 0.0;
  }
  double u = (m0 - x) * (m0 + x) / (m0 * m0);
  double g = x * std::sqrt(u) * std::exp(c * u);
  if (dg) {
    dg[0] = g * (0.5 / u + c) * 2.0 * x * x / (m0 * m0 * m0);
    dg[1] = g * u;
  }
  return g;
}

/* Johnson's S_U density (Sec. 3 names it among the built-in densities):
 * with z = (x - mu)/lambda and u = gamma + delta asinh(z),
 *   g = exp(-u^2/2) / sqrt(1 + z^2)
 * (the normalised density is delta/(lambda sqrt(2 pi)) g on the real line).
 * log g = -u^2/2 - ln(1 + z^2)/2, so with w = u delta/sqrt(1 + z^2) + z/(1 + z^2)
 * (which is -d log g/dz) and dz/dmu = -1/lambda, dz/dlambda = -z/lambda:
 *   dg/dmu = g w/lambda, dg/dlambda = g w z/lambda,
 *   dg/dgamma = -g u,    dg/ddelta = -g u asinh(z).                     */
double g_johnson(const orc_node& nd, const double* th, double x, double* dg) {
  double mu = P(th, nd, 0), la = P(th, nd, 1), ga = P(th, nd, 2), de = P(th, nd, 3);
  double z = (x - mu) / la;
  double q = 1.0 + z * z;
  double A = std::asinh(z);
  double u = ga + de * A;
  double g = std::exp(-0.5 * u * u) / std::sqrt(q);
  if (dg) {
    double w = u * de / std::sqrt(q) + z / q;
    dg[0] = g * w / la;
    dg[1] = g * w * z / la;
    dg[2] = -g * u;
    dg[3] = -g * u * A;
  }
  return g;
}

/* Chi-square with nu degrees of freedom (the "ChiSquarePdf" of Sec. 5.2's
 * benchmark): g = x^(nu/2 - 1) e^(-x/2) for x > 0; dg/dnu = g ln(x)/2. */
double g_chi2(const orc_node& nd, const double* th, double x, double* dg) {
  double nu = P(th, nd, 0);
  if (!(x >= 0.0)) {
    if (dg) dg[0] = 0.0;
    return 0.0;
  }
  double g = std::pow(x, 0.5 * nu - 1.0) * std::exp(-0.5 * x); /* at x = 0: 0, 1 or inf */
  if (dg) dg[0] = 0.5 * g * std::log(x);
  return g;
}

/* Hypatia2 (the two-sided Hypatia of Santos and Dupertuis, NIM A 764
 * (2014) 150, among the densities Sec. 3 adds to RooFit): a generalised
 * hyperbolic core of width sigma with power-law tails on both sides that
 * continue it with equal value and slope.  Parameters (mu, sigma, lambda,
 * zeta, beta, a_l, n_l, a_r, n_r); with d = x - mu, nu = lambda - 1/2,
 *   A^2 = zeta K_lambda(zeta) / K_{lambda+1}(zeta),  delta^2 = A^2 sigma^2,
 *   alpha = zeta / delta,  r = sqrt(d^2 + delta^2),
 *   core  G(d) = r^nu e^{beta d} K_nu(alpha r)          for -a_l sigma <= d <= a_r sigma,
 *   low   G_l (1 + s_l (d_l - d) / n_l)^{-n_l}           for d < d_l = -a_l sigma,
 *   high  G_h (1 - s_h (d - d_h) / n_r)^{-n_r}           for d > d_h = a_r sigma,
 * with G_l = G(d_l), s_l = G'(d_l)/G(d_l) > 0, G_h, s_h < 0 likewise.
 * K_nu is the modified Bessel function of the second kind, evaluated from
 * its integral K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt by the
 * trapezoidal rule (exponentially convergent for this analytic, doubly
 * exponentially decaying integrand).  Everything is templated on the
 * number type so that derivatives come from complex steps: for an analytic
 * f, f'(x) = Im f(x + i h) / h to rounding, with h tiny.                  */
using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }
inline double mag(double v) { return std::fabs(v); }
inline double mag(const cplx& v) { return std::abs(v); }

/* log K_nu(z), z > 0 (Re), from e^z K_nu(z) = int exp(-z (cosh t - 1)) cosh(nu t) dt. */
template <class T>
T log_bessel_k(T nu, T z) {
  const double zr = re(z);
  const double h = std::min(1.0 / 16.0, 0.25 / std::sqrt(zr));
  T sum = 0.5;  /* t = 0 */
  double prev = 1e300;
  for (int j = 1; j < 200000; ++j) {
    const double t = j * h;
    const T term = std::exp(-z * (std::cosh(t) - 1.0)) * std::cosh(nu * t);
    sum += term;
    const double a = mag(term);
    if (a < 1e-19 * mag(sum) && a <= prev) break;
    prev = a;
  }
  return std::log(h * sum) - z;
}

template <class T>
struct HypConst {
  T mu, nu, beta, delta2, alpha, dl, dh;
  T lGl, sl, nl, lGh, sh, nr;  /* junction values, log-slopes, exponents */
  bool ok;
};

/* log G and d log G / dd of the core at d */
template <class T>
void hyp_core(const HypConst<T>& c, T d, T* lg, T* slope) {
  const T r2 = d * d + c.delta2, r = std::sqrt(r2);
  const T z = c.alpha * r;
  const T lk = log_bessel_k(c.nu, z);
  *lg = 0.5 * c.nu * std::log(r2) + c.beta * d + lk;
  if (slope) {
    /* K_nu'(z) / K_nu(z) = nu / z - K_{nu+1}(z) / K_nu(z) */
    const T q = std::exp(log_bessel_k(c.nu + 1.0, z) - lk);
    *slope = 2.0 * c.nu * d / r2 + c.beta - c.alpha * (d / r) * q;
  }
}

template <class T>
HypConst<T> hyp_const(const T* p) {
  HypConst<T> c;
  const T mu = p[0], sg = p[1], la = p[2], ze = p[3], be = p[4];
  c.ok = re(sg) > 0.0 && re(ze) > 0.0 && re(p[5]) > 0.0 && re(p[6]) > 1.0 && re(p[7]) > 0.0 && re(p[8]) > 1.0;
  if (!c.ok) return c;
  c.mu = mu;
  c.nu = la - 0.5;
  c.beta = be;
  const T a2 = ze * std::exp(log_bessel_k(la, ze) - log_bessel_k(la + 1.0, ze));
  c.delta2 = a2 * sg * sg;
  c.alpha = ze / std::sqrt(c.delta2);
  c.dl = -p[5] * sg;
  c.dh = p[7] * sg;
  c.nl = p[6];
  c.nr = p[8];
  hyp_core(c, c.dl, &c.lGl, &c.sl);
  hyp_core(c, c.dh, &c.lGh, &c.sh);
  c.ok = re(c.sl) > 0.0 && re(c.sh) < 0.0;  /* tails must fall away from the core */
  return c;
}

/* log of the unnormalised density at d = x - mu */
template <class T>
T hyp_log_g(const HypConst<T>& c, T d) {
  if (re(d) < re(c.dl)) return c.lGl - c.nl * std::log(1.0 + c.sl * (c.dl - d) / c.nl);
  if (re(d) > re(c.dh)) return c.lGh - c.nr * std::log(1.0 - c.sh * (d - c.dh) / c.nr);
  T lg;
  hyp_core(c, d, &lg, (T*)nullptr);
  return lg;
}

/* int_{u}^{v} (1 + k w)^{-n} dw for 0 <= u <= v (a tail in the distance w
 * from its junction): ((1+kv)^{1-n} - (1+ku)^{1-n}) / (k (1-n)), by a
 * series in (1-n) log((1+kv)/(1+ku)) when n is close to 1 */
template <class T>
T tail_integral(T k, T n, T u, T v) {
  const T lu = std::log(1.0 + k * u), lv = std::log(1.0 + k * v);
  const T e = 1.0 - n;
  if (mag(e * (lv - lu)) > 1e-3) return (std::exp(e * lv) - std::exp(e * lu)) / (k * e);
  /* exp(e lu) (exp(e L) - 1) / (k e), L = lv - lu, by its series */
  const T L = lv - lu;
  T term = L, s = L;
  for (int j = 2; j < 30; ++j) {
    term *= e * L / (double)j;
    s += term;
  }
  return std::exp(e * lu) * s / k;
}

/* Z = int_lo^hi g dx (the density relative to the core's scale exp(lGl)) */
template <class T>
T hyp_norm(const HypConst<T>& c, double lo, double hi) {
  const T a = lo - c.mu, b = hi - c.mu;
  T Z = 0.0;
  /* low tail: d in [a, min(b, dl)], w = dl - d in [dl - min(b, dl), dl - a] */
  if (re(a) < re(c.dl)) {
    const T top = re(b) < re(c.dl) ? b : c.dl;
    Z += std::exp(c.lGl) * tail_integral(c.sl / c.nl, c.nl, c.dl - top, c.dl - a);
  }
  if (re(b) > re(c.dh)) {
    const T bot = re(a) > re(c.dh) ? a : c.dh;
    Z += std::exp(c.lGh) * tail_integral(-c.sh / c.nr, c.nr, bot - c.dh, b - c.dh);
  }
  /* core on [max(a, dl), min(b, dh)]: composite 256-point Gauss-Legendre on
   * 4 panels (peak width ~ sigma, core width (a_l + a_r) sigma) */
  const T ca = re(a) > re(c.dl) ? a : c.dl, cb = re(b) < re(c.dh) ? b : c.dh;
  if (re(cb) > re(ca)) {
    const Rule& R = rule256();
    const int npan = 4;
    for (int q = 0; q < npan; ++q) {
      const T pa = ca + (cb - ca) * ((double)q / npan), pb = ca + (cb - ca) * ((double)(q + 1) / npan);
      const T hw = 0.5 * (pb - pa), mid = 0.5 * (pa + pb);
      for (int i = 0; i < 256; ++i) {
        T lg;
        hyp_core(c, mid + hw * R.x[i], &lg, (T*)nullptr);
        Z += hw * R.w[i] * std::exp(lg);
      }
    }
  }
  return Z;
}

/* Per-parameter-point state of one Hypatia2 leaf: the constants at theta
 * and at theta + i h e_k for each of its 9 parameters, the reference log
 * value (the core at the left junction; every value and Z are taken
 * relative to it, which cancels in g / Z) and Z.  Cached per thread while
 * the parameters stay the same (events are processed one point at a time). */
constexpr int kHypNP = 9;
constexpr double kCstep = 1e-30;

struct HypPoint {
  double key[kHypNP];
  double lo, hi;
  bool valid = false;
  HypConst<double> c;
  HypConst<cplx> cc[kHypNP];
  cplx ref[kHypNP];
  double ref0;
  double Z;
  double dZ[kHypNP];
  bool ok;
};

const HypPoint& hyp_point(const orc_node& nd, const double* th, double lo, double hi) {
  thread_local HypPoint hp;
  bool same = hp.valid && hp.lo == lo && hp.hi == hi;
  for (int k = 0; k < kHypNP && same; ++k) same = hp.key[k] == P(th, nd, k);
  if (same) return hp;
  hp.valid = true;
  hp.lo = lo;
  hp.hi = hi;
  double p[kHypNP];
  for (int k = 0; k < kHypNP; ++k) hp.key[k] = p[k] = P(th, nd, k);
  hp.c = hyp_const<double>(p);
  hp.ok = hp.c.ok;
  if (!hp.ok) return hp;
  hp.ref0 = hp.c.lGl;
  hp.Z = hyp_norm(hp.c, lo, hi) * std::exp(-hp.ref0);
  for (int k = 0; k < kHypNP; ++k) {
    cplx pc[kHypNP];
    for (int j = 0; j < kHypNP; ++j) pc[j] = p[j];
    pc[k] += cplx(0.0, kCstep);
    hp.cc[k] = hyp_const<cplx>(pc);
    hp.ref[k] = hp.cc[k].lGl;
    hp.dZ[k] = (hyp_norm(hp.cc[k], lo, hi) * std::exp(-hp.ref[k])).imag() / kCstep;
  }
  return hp;
}

/* g relative to the reference value, and dg / dtheta_local by complex steps */
double g_hypatia(const orc_model& m, const orc_node& nd, const double* th, double x, double* dg) {
  const HypPoint& hp = hyp_point(nd, th, m.lo[nd.obs], m.hi[nd.obs]);
  if (!hp.ok) {
    if (dg)
      for (int k = 0; k < kHypNP; ++k) dg[k] = 0.0;
    return std::nan("");
  }
  const double lg = hyp_log_g(hp.c, x - hp.c.mu) - hp.ref0;
  const double g = std::exp(lg);
  if (dg)
    for (int k = 0; k < kHypNP; ++k) {
      const cplx l = hyp_log_g(hp.cc[k], cplx(x) - hp.cc[k].mu) - hp.ref[k];
      dg[k] = g * l.imag() / kCstep;
    }
  return g;
}

void norm_hypatia(const orc_model& m, const orc_node& nd, const double* th, double* Z, double* d) {
  const HypPoint& hp = hyp_point(nd, th, m.lo[nd.obs], m.hi[nd.obs]);
  if (!hp.ok) {
    *Z = std::nan("");
    return;
  }
  *Z = hp.Z;
  for (int k = 0; k < kHypNP; ++k) d[k] = hp.dZ[k];
}

double leaf_g(const orc_model& m, const orc_node& nd, const double* th, double x, double* dg) {
  switch (nd.kind) {
    case ORC_GAUSS: return g_gauss(nd, th, x, dg);
    case ORC_EXP: return g_exp(nd, th, x, dg);
    case ORC_CHEB: return g_cheb(nd, th, m.lo[nd.obs], m.hi[nd.obs], x, dg);
    case ORC_CB: return g_cb(nd, th, x, dg);
    case ORC_ARGUS: return g_argus(nd, th, x, dg);
    case ORC_JOHNSON: return g_johnson(nd, th, x, dg);
    case ORC_CHI2: return g_chi2(nd, th, x, dg);
    case ORC_HYPATIA: return g_hypatia(m, nd, th, x, dg);
  }
  return std::nan("");
}

/* ------------------------------------------------------------------ */
/* Normalisation integrals.                                             */
/* ------------------------------------------------------------------ */

/* erf(b/sqrt2) - erf(a/sqrt2) for a <= b, using erfc when both are on the
 * same side of zero (avoids cancellation in the far tails). */
double erf_diff(double a, double b) {
  const double r = 1.0 / std::sqrt(2.0);
  if (a >= 0.0) return std::erfc(a * r) - std::erfc(b * r);
  if (b <= 0.0) return std::erfc(-b * r) - std::erfc(-a * r);
  return std::erf(b * r) - std::erf(a * r);
}

/* Gaussian over [lo, hi]: Z = sigma sqrt(pi/2) [erf(b/sqrt2) - erf(a/sqrt2)]
 * with a, b the standardised limits; derivatives by differentiating under
 * the integral sign:
 *   dZ/dmu    = e^{-a^2/2} - e^{-b^2/2}
 *   dZ/dsigma = Z/sigma + a e^{-a^2/2} - b e^{-b^2/2}.                  */
void norm_gauss_closed(double mu, double s, double lo, double hi, double* Z, double* d) {
  double a = (lo - mu) / s, b = (hi - mu) / s;
  double ea = std::exp(-0.5 * a * a), eb = std::exp(-0.5 * b * b);
  double z = s * std::sqrt(kPi / 2.0) * erf_diff(a, b);
  *Z = z;
  d[0] = ea - eb;
  d[1] = z / s + a * ea - b * eb;
}

/* Exponential over [lo, hi]: Z = int e^{cx} dx, dZ/dc = int x e^{cx} dx.
 * Power series in c when |c| max(|lo|,|hi|) is small, else closed form. */
void norm_exp_closed(double c, double lo, double hi, double* Z, double* d) {
  double R = std::max(std::fabs(lo), std::fabs(hi));
  if (std::fabs(c) * R < 0.5) {
    Neumaier z, dz;
    double ck = 1.0; /* c^k / k! */
    double hp = hi, lp = lo;
    for (int k = 0; k < 60; ++k) {
      /* hp = hi^{k+1}, lp = lo^{k+1} */
      z.add(ck * (hp - lp) / (k + 1));
      dz.add(ck * (hp * hi - lp * lo) / (k + 2));
      hp *= hi;
      lp *= lo;
      ck *= c / (k + 1);
    }
    *Z = z.value();
    d[0] = dz.value();
    return;
  }
  double ehi = std::exp(c * hi), elo = std::exp(c * lo);
  double z = elo * std::expm1(c * (hi - lo)) / c;
  *Z = z;
  d[0] = (ehi * (c * hi - 1.0) - elo * (c * lo - 1.0)) / (c * c);
}

/* Chebyshev: int_{-1}^{1} T_k = 2/(1-k^2) for even k, 0 for odd k. */
void norm_cheb_closed(const orc_node& nd, const double* th, double lo, double hi, double* Z,
                      double* d) {
  double h = hi - lo;
  double z = h; /* T_0 term: (hi-lo)/2 * 2 */
  for (int k = 1; k <= nd.n_param; ++k) {
    double ik = (k % 2 == 0) ? 2.0 / (1.0 - (double)k * k) : 0.0;
    z += 0.5 * h * P(th, nd, k - 1) * ik;
    d[k - 1] = 0.5 * h * ik;
  }
  *Z = z;
}

/* Crystal Ball closed form.  Core piece over t in [ca, cb], tail piece over
 * t in [ta, tb] (t = (m - m0)/sigma, dm = sigma dt, D = B - t):
 *   core: sigma sqrt(pi/2) [erf]                       (as the Gaussian)
 *   tail: sigma A/(n-1) [D^{1-n}]                        since
 *         int D^{-n} dt = D^{1-n}/(n-1), int D^{-n-1} dt = D^{-n}/n,
 *         int D^{-n} ln D dt = D^{1-n} (ln D/(n-1) + 1/(n-1)^2).
 * Derivatives are int dg/dtheta dm over the fixed m-range (g is continuous
 * at the junction, so the moving split point contributes nothing).      */
void norm_cb_closed(double m0, double s, double a, double n, double lo, double hi, double* Z,
                    double* d) {
  double tlo = (lo - m0) / s, thi = (hi - m0) / s;
  double z = 0.0;
  d[0] = d[1] = d[2] = d[3] = 0.0;
  double ca = std::max(tlo, -a), cb = thi;
  if (cb > ca) {
    double ea = std::exp(-0.5 * ca * ca), eb = std::exp(-0.5 * cb * cb);
    double zc = s * std::sqrt(kPi / 2.0) * erf_diff(ca, cb);
    z += zc;
    d[0] += ea - eb;
    d[1] += zc / s + ca * ea - cb * eb;
  }
  double ta = tlo, tb = std::min(thi, -a);
  if (tb > ta) {
    double A = std::pow(n / a, n) * std::exp(-0.5 * a * a);
    double B = n / a - a;
    double Da = B - ta, Db = B - tb;
    auto F = [n](double D) {
      return std::pow(D, 1.0 - n) * (std::log(D) / (n - 1.0) + 1.0 / ((n - 1.0) * (n - 1.0)));
    };
    double dDn = std::pow(Db, -n) - std::pow(Da, -n);          /* [D^{-n}]     */
    double dD1n = std::pow(Db, 1.0 - n) - std::pow(Da, 1.0 - n); /* [D^{1-n}]   */
    double zt = s * A / (n - 1.0) * dD1n;
    z += zt;
    d[0] += -A * dDn;
    d[1] += -n * A * (B * dDn / n - dD1n / (n - 1.0));
    d[2] += (-n / a - a) * zt + (n / (a * a) + 1.0) * s * A * dDn;
    d[3] += (std::log(n / a) + 1.0) * zt - s * A * (F(Db) - F(Da)) - s * A * dDn / a;
  }
  *Z = z;
}

/* J_p(U) = int_0^U u^p e^{c u} du for p > -1, by series with positive
 * terms only:
 *   c >= 0: U^{p+1} sum_j (cU)^j / (j! (j + p + 1))
 *   c <  0: U^{p+1} e^{-kU} sum_j (kU)^j / prod_{i=0..j} (p + 1 + i), k = -c
 * (the second is the series of the lower incomplete gamma function). */
double J_series(double p, double c, double U) {
  if (U <= 0.0) return 0.0;
  double a = p + 1.0;
  Neumaier sum;
  if (c >= 0.0) {
    double x = c * U, term = 1.0; /* x^j / j! */
    for (int j = 0; j < 5000; ++j) {
      double add = term / (j + a);
      sum.add(add);
      if (j > 2 && add < 1e-19 * sum.value()) break;
      term *= x / (j + 1);
    }
    return std::pow(U, a) * sum.value();
  }
  double x = -c * U, term = 1.0 / a;
  for (int j = 0; j < 5000; ++j) {
    sum.add(term);
    if (j > 2 && term < 1e-19 * sum.value()) break;
    term *= x / (a + j + 1);
  }
  return std::pow(U, a) * std::exp(-x) * sum.value();
}

/* ARGUS over [lo, min(hi, m0)] in the variable u = 1 - (m/m0)^2
 * (m dm = -m0^2/2 du):
 *   Z      = m0^2/2 [J_{1/2}]
 *   dZ/dc  = m0^2/2 [J_{3/2}]
 *   dZ/dm0 = m0 [ (J_{-1/2} - J_{1/2})/2 + c (J_{1/2} - J_{3/2}) ]
 * each bracket taken between u(lo) and u(min(hi, m0)).                 */
void norm_argus_closed(double m0, double c, double lo, double hi, double* Z, double* d) {
  double Ua = (m0 - lo) * (m0 + lo) / (m0 * m0);
  double Ub = (hi >= m0) ? 0.0 : (m0 - hi) * (m0 + hi) / (m0 * m0);
  auto J = [c, Ua, Ub](double p) { return J_series(p, c, Ua) - J_series(p, c, Ub); };
  double jm = J(-0.5), j1 = J(0.5), j3 = J(1.5);
  *Z = 0.5 * m0 * m0 * j1;
  d[0] = m0 * (0.5 * (jm - j1) + c * (j1 - j3));
  d[1] = 0.5 * m0 * m0 * j3;
}

/* Johnson S_U over [lo, hi].  The substitution u = gamma + delta asinh(z),
 * du = delta dx / (lambda sqrt(1 + z^2)), turns g dx into
 * (lambda/delta) e^{-u^2/2} du, so
 *   Z = (lambda/delta) sqrt(pi/2) [erf(u_hi/sqrt2) - erf(u_lo/sqrt2)].
 * Derivatives: the prefactor's, plus e^{-u^2/2} times the derivative of
 * each limit u_b (du_b/dmu = -delta/(lambda s_b), du_b/dlambda =
 * -delta z_b/(lambda s_b), du_b/dgamma = 1, du_b/ddelta = asinh(z_b), with
 * s_b = sqrt(1 + z_b^2)), taken between lo and hi:
 *   dZ/dmu     = e_lo/s_lo - e_hi/s_hi
 *   dZ/dlambda = Z/lambda + z_lo e_lo/s_lo - z_hi e_hi/s_hi
 *   dZ/dgamma  = (lambda/delta) (e_hi - e_lo)
 *   dZ/ddelta  = -Z/delta + (lambda/delta) (A_hi e_hi - A_lo e_lo).       */
void norm_johnson_closed(double mu, double la, double ga, double de, double lo, double hi,
                         double* Z, double* d) {
  double zl = (lo - mu) / la, zh = (hi - mu) / la;
  double Al = std::asinh(zl), Ah = std::asinh(zh);
  double ul = ga + de * Al, uh = ga + de * Ah;
  double sl = std::sqrt(1.0 + zl * zl), sh = std::sqrt(1.0 + zh * zh);
  double el = std::exp(-0.5 * ul * ul), eh = std::exp(-0.5 * uh * uh);
  double k = la / de;
  double z = k * std::sqrt(kPi / 2.0) * erf_diff(ul, uh);
  *Z = z;
  d[0] = el / sl - eh / sh;
  d[1] = z / la + zl * el / sl - zh * eh / sh;
  d[2] = k * (eh - el);
  d[3] = -z / de + k * (Ah * eh - Al * el);
}

/* Lower incomplete gamma function gamma(k, y) = int_0^y t^(k-1) e^(-t) dt
 * and its derivative in k, from the series
 *   gamma(k, y) = y^k e^(-y) sum_{n>=0} y^n / (k (k+1) ... (k+n))
 * (all terms positive); differentiating each term in k gives
 *   d gamma/dk = gamma ln y - y^k e^(-y) sum_n t_n H_n,
 * t_n the n-th term, H_n = sum_{j=0..n} 1/(k+j).  y^k e^(-y) is formed as
 * exp(k ln y - y) after the sum, so that y up to ~700 neither over- nor
 * underflows.  gamma(k, 0) = 0 and its k-derivative is 0 (k > 0). */
void lower_gamma(double k, double y, double* g, double* dg) {
  *g = 0.0;
  *dg = 0.0;
  if (!(y > 0.0)) return;
  Neumaier S, D;
  double t = 1.0 / k, H = 1.0 / k;
  for (int n = 0; n < 100000; ++n) {
    S.add(t);
    D.add(t * H);
    if (n > y && t < 1e-19 * S.value()) break;
    t *= y / (k + n + 1);
    H += 1.0 / (k + n + 1);
  }
  double pre = std::exp(k * std::log(y) - y);
  *g = pre * S.value();
  *dg = *g * std::log(y) - pre * D.value();
}

/* Chi-square over [lo, hi], lo >= 0: with x = 2t and k = nu/2,
 *   Z = int x^(k-1) e^(-x/2) dx = 2^k [gamma(k, hi/2) - gamma(k, lo/2)],
 *   dZ/dnu = (1/2) dZ/dk = (1/2) { ln2 Z + 2^k [gamma'(k, hi/2) - gamma'(k, lo/2)] }
 * (gamma' the k-derivative).  Both ends are evaluated separately, so a
 * range that starts deep in the upper tail loses digits to cancellation;
 * there the Gauss-Legendre rule (the integrand is analytic for lo > 0) is
 * the accurate choice. */
void norm_chi2_closed(double nu, double lo, double hi, double* Z, double* d) {
  double k = 0.5 * nu;
  double ga, dga, gb, dgb;
  lower_gamma(k, 0.5 * lo, &ga, &dga);
  lower_gamma(k, 0.5 * hi, &gb, &dgb);
  double p2 = std::exp2(k);
  double z = p2 * (gb - ga);
  *Z = z;
  d[0] = 0.5 * (std::log(2.0) * z + p2 * (dgb - dga));
}

/* 256-point Gauss-Legendre on [a, b] of g and dg (np local derivatives). */
void gl_panel(const orc_model& m, const orc_node& nd, const double* th, double a, double b,
              double* Z, double* d) {
  const Rule& r = rule256();
  double h = 0.5 * (b - a), c = 0.5 * (a + b);
  double dg[ORC_NODE_PAR];
  for (size_t i = 0; i < r.x.size(); ++i) {
    double x = c + h * r.x[i];
    double g = leaf_g(m, nd, th, x, dg);
    *Z += h * r.w[i] * g;
    for (int k = 0; k < nd.n_param; ++k) d[k] += h * r.w[i] * dg[k];
  }
}

/* ARGUS after m = m0 - s^2 (dm = 2 s ds), which makes the integrand
 * analytic in s; u = s^2 (2 m0 - s^2)/m0^2 is formed from s directly. */
void gl_argus_subst(const orc_node& nd, const double* th, double lo, double hi, double* Z,
                    double* d) {
  double m0 = P(th, nd, 0), c = P(th, nd, 1);
  double sa = std::sqrt(m0 - std::min(hi, m0)), sb = std::sqrt(m0 - lo);
  const Rule& r = rule256();
  double h = 0.5 * (sb - sa), cc = 0.5 * (sa + sb);
  for (size_t i = 0; i < r.x.size(); ++i) {
    double sv = cc + h * r.x[i];
    double mm = m0 - sv * sv;
    double u = sv * sv * (2.0 * m0 - sv * sv) / (m0 * m0);
    double g = mm * std::sqrt(u) * std::exp(c * u);
    double jac = 2.0 * sv * h * r.w[i];
    *Z += jac * g;
    d[0] += jac * g * (0.5 / u + c) * 2.0 * mm * mm / (m0 * m0 * m0);
    d[1] += jac * g * u;
  }
}

/* Chi-square on [0, hi] after x = s^2 (dx = 2 s ds): the integrand
 * 2 s^(nu-1) e^(-s^2/2) is a polynomial times a Gaussian for integer nu
 * (and smooth enough for 256 nodes to reach double precision for
 * nu >~ 3 otherwise); dg/dnu = g ln s. */
void gl_chi2_subst(const orc_node& nd, const double* th, double hi, double* Z, double* d) {
  double nu = P(th, nd, 0);
  const Rule& r = rule256();
  double sb = std::sqrt(hi);
  double h = 0.5 * sb, cc = 0.5 * sb;
  for (size_t i = 0; i < r.x.size(); ++i) {
    double sv = cc + h * r.x[i];
    double g = 2.0 * std::pow(sv, nu - 1.0) * std::exp(-0.5 * sv * sv);
    *Z += h * r.w[i] * g;
    d[0] += h * r.w[i] * g * std::log(sv);
  }
}

/* Z and dZ (local parameter order) of one leaf. */
void leaf_norm_local(const orc_model& m, const orc_node& nd, const double* th, double* Z,
                     double* d) {
  double lo = m.lo[nd.obs], hi = m.hi[nd.obs];
  *Z = 0.0;
  for (int k = 0; k < ORC_NODE_PAR; ++k) d[k] = 0.0;
  if (nd.kind == ORC_HYPATIA) { /* tails in closed form, the core by quadrature, any norm flag */
    norm_hypatia(m, nd, th, Z, d);
    return;
  }
  if (nd.norm == ORC_NORM_CLOSED) {
    switch (nd.kind) {
      case ORC_GAUSS: norm_gauss_closed(P(th, nd, 0), P(th, nd, 1), lo, hi, Z, d); return;
      case ORC_EXP: norm_exp_closed(P(th, nd, 0), lo, hi, Z, d); return;
      case ORC_CHEB: norm_cheb_closed(nd, th, lo, hi, Z, d); return;
      case ORC_CB:
        norm_cb_closed(P(th, nd, 0), P(th, nd, 1), P(th, nd, 2), P(th, nd, 3), lo, hi, Z, d);
        return;
      case ORC_ARGUS: norm_argus_closed(P(th, nd, 0), P(th, nd, 1), lo, hi, Z, d); return;
      case ORC_JOHNSON:
        norm_johnson_closed(P(th, nd, 0), P(th, nd, 1), P(th, nd, 2), P(th, nd, 3), lo, hi, Z, d);
        return;
      case ORC_CHI2: norm_chi2_closed(P(th, nd, 0), lo, hi, Z, d); return;
    }
    return;
  }
  if (nd.norm == ORC_NORM_GL_SINGLE) {
    gl_panel(m, nd, th, lo, hi, Z, d);
    return;
  }
  /* ORC_NORM_GL_SPLIT */
  if (nd.kind == ORC_CB) {
    double mj = P(th, nd, 0) - P(th, nd, 2) * P(th, nd, 1);
    if (mj <= lo || mj >= hi) {
      gl_panel(m, nd, th, lo, hi, Z, d);
    } else {
      gl_panel(m, nd, th, lo, mj, Z, d);
      gl_panel(m, nd, th, mj, hi, Z, d);
    }
    return;
  }
  if (nd.kind == ORC_ARGUS) {
    gl_argus_subst(nd, th, lo, hi, Z, d);
    return;
  }
  if (nd.kind == ORC_CHI2 && lo == 0.0) {
    gl_chi2_subst(nd, th, hi, Z, d);
    return;
  }
  gl_panel(m, nd, th, lo, hi, Z, d);
}

/* ------------------------------------------------------------------ */
/* Model checks.                                                        */
/* ------------------------------------------------------------------ */
int expected_params(const orc_node& nd) {
  switch (nd.kind) {
    case ORC_GAUSS: return 2;
    case ORC_EXP: return 1;
    case ORC_CHEB: return (nd.n_param >= 1 && nd.n_param <= ORC_NODE_PAR) ? nd.n_param : -1;
    case ORC_CB: return 4;
    case ORC_ARGUS: return 2;
    case ORC_SUM: return (nd.n_param == nd.n_child) ? nd.n_child : nd.n_child - 1;
    case ORC_PROD: return 0;
    case ORC_JOHNSON: return 4;
    case ORC_CHI2: return 1;
    case ORC_HYPATIA: return 9;
  }
  return -1;
}

/* A SUM with one coefficient per child takes them as yields. */
bool sum_of_yields(const orc_node& nd) { return nd.kind == ORC_SUM && nd.n_param == nd.n_child; }

/* The SUM whose yields make the expected event count of an extended model
 * without a separate yield parameter: the root if it is a sum of yields,
 * else the one sum of yields among the children of a root product; -1 if
 * there is none (or more than one). */
int extended_sum(const orc_model& m) {
  const orc_node& r = m.node[m.root];
  if (sum_of_yields(r)) return m.root;
  if (r.kind != ORC_PROD) return -1;
  int found = -1;
  for (int j = 0; j < r.n_child; ++j) {
    if (sum_of_yields(m.node[r.child[j]])) {
      if (found >= 0) return -1;
      found = r.child[j];
    }
  }
  return found;
}

/* Parameter k enters the expected event count of an extended model. */
bool is_yield(const orc_model& m, int k) {
  if (m.yield_param >= 0) return k == m.yield_param;
  const orc_node& s = m.node[extended_sum(m)];
  for (int q = 0; q < s.n_param; ++q)
    if (s.param[q] == k) return true;
  return false;
}

/* The expected event count nu of an extended model at theta. */
double total_yield(const orc_model& m, const double* th) {
  if (m.yield_param >= 0) return th[m.yield_param];
  const orc_node& s = m.node[extended_sum(m)];
  double nu = 0.0;
  for (int k = 0; k < s.n_param; ++k) nu += th[s.param[k]];
  return nu;
}

bool is_leaf(int kind) {
  return (kind >= ORC_GAUSS && kind <= ORC_ARGUS) || kind == ORC_JOHNSON || kind == ORC_CHI2 || kind == ORC_HYPATIA;
}

/* Bit mask of observables a node depends on. */
unsigned obs_mask(const orc_model& m, int i) {
  const orc_node& nd = m.node[i];
  if (is_leaf(nd.kind)) return 1u << nd.obs;
  unsigned r = 0;
  for (int j = 0; j < nd.n_child; ++j) r |= obs_mask(m, nd.child[j]);
  return r;
}

int check_model(const orc_model& m) {
  if (m.n_obs < 1 || m.n_obs > ORC_MAX_OBS) return ORC_E_ARG;
  if (m.n_param < 0 || m.n_param > ORC_MAX_PAR) return ORC_E_ARG;
  if (m.n_node < 1 || m.n_node > ORC_MAX_NODE) return ORC_E_ARG;
  if (m.root < 0 || m.root >= m.n_node) return ORC_E_ARG;
  for (int o = 0; o < m.n_obs; ++o)
    if (!(m.lo[o] < m.hi[o])) return ORC_E_ARG;
  for (int i = 0; i < m.n_node; ++i) {
    const orc_node& nd = m.node[i];
    if (nd.kind < ORC_GAUSS || nd.kind > ORC_HYPATIA) return ORC_E_ARG;
    if (nd.n_param < 0 || nd.n_param > ORC_NODE_PAR) return ORC_E_ARG;
    if (expected_params(nd) != nd.n_param) return ORC_E_ARG;
    for (int k = 0; k < nd.n_param; ++k)
      if (nd.param[k] < 0 || nd.param[k] >= m.n_param) return ORC_E_ARG;
    if (is_leaf(nd.kind)) {
      if (nd.obs < 0 || nd.obs >= m.n_obs || nd.n_child != 0) return ORC_E_ARG;
      if (nd.norm < ORC_NORM_CLOSED || nd.norm > ORC_NORM_GL_SINGLE) return ORC_E_ARG;
      if (nd.kind == ORC_ARGUS && m.lo[nd.obs] < 0.0) return ORC_E_UNSUPPORTED;
      if (nd.kind == ORC_CHI2 && (m.lo[nd.obs] < 0.0 || m.hi[nd.obs] > 1000.0)) return ORC_E_UNSUPPORTED;
    } else {
      if (nd.n_child < (nd.kind == ORC_SUM ? 2 : 1) || nd.n_child > ORC_NODE_CHILD)
        return ORC_E_ARG;
      for (int j = 0; j < nd.n_child; ++j)
        if (nd.child[j] < 0 || nd.child[j] >= i) return ORC_E_ARG; /* topological */
      if (nd.kind == ORC_SUM) {
        unsigned m0 = obs_mask(m, nd.child[0]);
        for (int j = 1; j < nd.n_child; ++j)
          if (obs_mask(m, nd.child[j]) != m0) return ORC_E_UNSUPPORTED;
      } else {
        unsigned seen = 0;
        for (int j = 0; j < nd.n_child; ++j) {
          unsigned mk = obs_mask(m, nd.child[j]);
          if (mk & seen) return ORC_E_UNSUPPORTED; /* products over disjoint observables */
          seen |= mk;
        }
      }
    }
  }
  if (obs_mask(m, m.root) != (1u << m.n_obs) - 1u) return ORC_E_UNSUPPORTED;
  if (m.extended) {
    if (m.yield_param >= m.n_param) return ORC_E_ARG;
    if (m.yield_param < 0 && extended_sum(m) < 0) return ORC_E_ARG;
  }
  return ORC_OK;
}

/* Parameter-range checks of Sec. 3: declared [lo, hi] per parameter plus
 * the constraints of each density. */
int check_params(const orc_model& m, const double* th) {
  for (int k = 0; k < m.n_param; ++k) {
    if (!(th[k] >= m.par_lo[k] && th[k] <= m.par_hi[k])) return ORC_E_PARAM; /* NaN too */
  }
  for (int i = 0; i < m.n_node; ++i) {
    const orc_node& nd = m.node[i];
    switch (nd.kind) {
      case ORC_GAUSS:
        if (!(P(th, nd, 1) > 0.0)) return ORC_E_PARAM;
        break;
      case ORC_CB:
        if (!(P(th, nd, 1) > 0.0) || !(P(th, nd, 2) > 0.0) || !(P(th, nd, 3) > 1.0))
          return ORC_E_PARAM;
        break;
      case ORC_ARGUS:
        if (!(P(th, nd, 0) > m.lo[nd.obs])) return ORC_E_PARAM;
        break;
      case ORC_JOHNSON:
        if (!(P(th, nd, 1) > 0.0) || !(P(th, nd, 3) > 0.0)) return ORC_E_PARAM;
        break;
      case ORC_CHI2:
        if (!(P(th, nd, 0) > 0.0)) return ORC_E_PARAM;
        break;
      case ORC_HYPATIA: /* sigma, zeta, a_l, a_r > 0, n_l, n_r > 1, and tails that fall */
        if (!hyp_point(nd, th, m.lo[nd.obs], m.hi[nd.obs]).ok) return ORC_E_PARAM;
        break;
      case ORC_SUM: {
        double f = 0.0;
        if (sum_of_yields(nd)) { /* yields >= 0 with a positive total */
          for (int k = 0; k < nd.n_param; ++k) {
            double v = P(th, nd, k);
            if (!(v >= 0.0)) return ORC_E_PARAM;
            f += v;
          }
          if (!(f > 0.0) || !std::isfinite(f)) return ORC_E_PARAM;
          break;
        }
        for (int k = 0; k < nd.n_param; ++k) {
          double v = P(th, nd, k);
          if (!(v >= 0.0 && v <= 1.0)) return ORC_E_PARAM;
          f += v;
        }
        if (!(f <= 1.0)) return ORC_E_PARAM;
        break;
      }
      default: break;
    }
  }
  if (m.extended && !(total_yield(m, th) > 0.0)) return ORC_E_PARAM;
  return ORC_OK;
}

/* Per-parameter-point cache: the normalisation of every leaf. */
struct Prepared {
  const orc_model* m;
  const double* th;
  double Z[ORC_MAX_NODE];
  double dZ[ORC_MAX_NODE][ORC_NODE_PAR]; /* local order */
};

int prepare(const orc_model& m, const double* th, Prepared& pr) {
  pr.m = &m;
  pr.th = th;
  int st = check_params(m, th);
  if (st != ORC_OK) return st;
  for (int i = 0; i < m.n_node; ++i) {
    const orc_node& nd = m.node[i];
    if (!is_leaf(nd.kind)) continue;
    leaf_norm_local(m, nd, th, &pr.Z[i], pr.dZ[i]);
    if (!(pr.Z[i] > 0.0) || !std::isfinite(pr.Z[i])) return ORC_E_PARAM;
  }
  return ORC_OK;
}

/* Value of node i at event x and, if dv != NULL, d value / d theta over all
 * n_param parameters. */
double node_value(const Prepared& pr, int i, const double* x, double* dv) {
  const orc_model& m = *pr.m;
  const orc_node& nd = m.node[i];
  const int np = m.n_param;
  if (is_leaf(nd.kind)) {
    double dg[ORC_NODE_PAR];
    double g = leaf_g(m, nd, pr.th, x[nd.obs], dv ? dg : nullptr);
    double Z = pr.Z[i];
    double v = g / Z;
    if (dv) {
      for (int k = 0; k < np; ++k) dv[k] = 0.0;
      /* d(g/Z) = dg/Z - g dZ / Z^2 */
      for (int k = 0; k < nd.n_param; ++k) dv[nd.param[k]] += dg[k] / Z - g * pr.dZ[i][k] / (Z * Z);
    }
    return v;
  }
  double cd[ORC_MAX_PAR];
  if (sum_of_yields(nd)) {
    /* p = sum_j nu_j p_j / S, S = sum_j nu_j; d p / d nu_j = (p_j - p) / S */
    double S = 0.0;
    for (int k = 0; k < nd.n_param; ++k) S += P(pr.th, nd, k);
    double v = 0.0;
    double vals[ORC_NODE_CHILD];
    if (dv)
      for (int k = 0; k < np; ++k) dv[k] = 0.0;
    for (int j = 0; j < nd.n_child; ++j) {
      vals[j] = node_value(pr, nd.child[j], x, dv ? cd : nullptr);
      double coef = P(pr.th, nd, j) / S;
      v += coef * vals[j];
      if (dv)
        for (int k = 0; k < np; ++k) dv[k] += coef * cd[k];
    }
    if (dv)
      for (int j = 0; j < nd.n_child; ++j) dv[nd.param[j]] += (vals[j] - v) / S;
    return v;
  }
  if (nd.kind == ORC_SUM) {
    double v = 0.0, flast = 1.0;
    if (dv)
      for (int k = 0; k < np; ++k) dv[k] = 0.0;
    for (int k = 0; k < nd.n_param; ++k) flast -= P(pr.th, nd, k);
    for (int j = 0; j < nd.n_child; ++j) {
      double cv = node_value(pr, nd.child[j], x, dv ? cd : nullptr);
      double coef = (j < nd.n_child - 1) ? P(pr.th, nd, j) : flast;
      v += coef * cv;
      if (dv) {
        for (int k = 0; k < np; ++k) dv[k] += coef * cd[k];
        if (j < nd.n_child - 1) {
          dv[nd.param[j]] += cv;
        } else {
          for (int q = 0; q < nd.n_param; ++q) dv[nd.param[q]] -= cv;
        }
      }
    }
    return v;
  }
  /* ORC_PROD */
  double v = 1.0;
  double vals[ORC_NODE_CHILD];
  double dchild[ORC_NODE_CHILD][ORC_MAX_PAR];
  for (int j = 0; j < nd.n_child; ++j) {
    vals[j] = node_value(pr, nd.child[j], x, dv ? dchild[j] : nullptr);
    v *= vals[j];
  }
  if (dv) {
    for (int k = 0; k < np; ++k) dv[k] = 0.0;
    for (int j = 0; j < nd.n_child; ++j) {
      double others = 1.0;
      for (int q = 0; q < nd.n_child; ++q)
        if (q != j) others *= vals[q];
      for (int k = 0; k < np; ++k) dv[k] += others * dchild[j][k];
    }
  }
  return v;
}

struct Partial {
  Neumaier nll;
  Neumaier grad[ORC_MAX_PAR];
  Neumaier abs_l;
  Neumaier abs_g[ORC_MAX_PAR];
  Neumaier wsum;                /* sum of the events' weights */
  std::vector<Neumaier> outer;  // n_param^2 when the BHHH matrix is wanted
  int status = ORC_OK;
};

/* Events [b, e).  w (may be NULL: every weight 1): per-event weights; the
 * event's log-density and its derivatives enter multiplied by w_i. */
void nll_range(const Prepared& pr, const double* const* cols, const double* w, int64_t b, int64_t e,
               bool want_grad, Partial& out) {
  const bool want_outer = !out.outer.empty();
  const orc_model& m = *pr.m;
  const int np = m.n_param;
  double x[ORC_MAX_OBS];
  double dv[ORC_MAX_PAR];
  for (int64_t i = b; i < e; ++i) {
    for (int o = 0; o < m.n_obs; ++o) {
      x[o] = cols[o][i];
      if (!(x[o] >= m.lo[o] && x[o] <= m.hi[o])) {
        out.status = ORC_E_DOMAIN;
        return;
      }
    }
    double p = node_value(pr, m.root, x, want_grad ? dv : nullptr);
    if (!(p > 0.0) || !std::isfinite(p)) {
      out.status = ORC_E_PDF;
      return;
    }
    double l = std::log(p);
    double wi = w ? w[i] : 1.0;
    out.nll.add(-wi * l);
    out.abs_l.add(std::fabs(wi * l));
    out.wsum.add(wi);
    if (want_grad) {
      double dl[ORC_MAX_PAR];
      for (int k = 0; k < np; ++k) {
        dl[k] = dv[k] / p; /* d log p = dp / p */
        out.grad[k].add(-wi * dl[k]);
        out.abs_g[k].add(std::fabs(wi * dl[k]));
      }
      /* BHHH: the outer product of the event's score with itself */
      if (want_outer)
        for (int j = 0; j < np; ++j)
          for (int k = j; k < np; ++k) out.outer[(size_t)j * np + k].add(dl[j] * dl[k]);
    }
  }
}

/* One dataset, one parameter point.  bhhh (may be NULL): the n_param x
 * n_param matrix sum_i s_i s_i^T of the events' scores s_i = d log p(x_i)
 * / d theta (symmetric, row-major), plus the Poisson term's own second
 * derivative N / nu^2 at (nu, nu) in an extended model; rows and columns of
 * fixed parameters are 0. */
int nll_one(const orc_model& m, const double* const* cols, int64_t n, const double* th,
            int threads, double* nll, double* grad, double* stats, double* bhhh = nullptr,
            const double* w = nullptr, double* wsum_out = nullptr) {
  const int np = m.n_param;
  auto fail = [&](int st) {
    *nll = kInf;
    if (grad)
      for (int k = 0; k < np; ++k) grad[k] = 0.0;
    if (bhhh)
      for (int k = 0; k < np * np; ++k) bhhh[k] = 0.0;
    return st;
  };
  Prepared pr;
  int st = prepare(m, th, pr);
  if (st != ORC_OK) return fail(st);
  int T = std::max(1, threads);
  if (n < 4096) T = 1;
  std::vector<Partial> parts(T);
  if (bhhh)
    for (auto& pt : parts) pt.outer.resize((size_t)np * np);
  const bool want_grad = (grad != nullptr) || (stats != nullptr) || (bhhh != nullptr);
  if (T == 1) {
    nll_range(pr, cols, w, 0, n, want_grad, parts[0]);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t) {
      int64_t b = n * t / T, e = n * (t + 1) / T;
      pool.emplace_back([&, b, e, t]() { nll_range(pr, cols, w, b, e, want_grad, parts[t]); });
    }
    for (auto& th_ : pool) th_.join();
  }
  /* fixed-order combine of the per-chunk compensated sums */
  Neumaier tot, g[ORC_MAX_PAR], al, ag[ORC_MAX_PAR], ws;
  for (int t = 0; t < T; ++t) {
    if (parts[t].status != ORC_OK) return fail(parts[t].status);
    tot.add(parts[t].nll.s);
    tot.add(parts[t].nll.c);
    ws.add(parts[t].wsum.s);
    ws.add(parts[t].wsum.c);
    al.add(parts[t].abs_l.s);
    al.add(parts[t].abs_l.c);
    for (int k = 0; k < np; ++k) {
      g[k].add(parts[t].grad[k].s);
      g[k].add(parts[t].grad[k].c);
      ag[k].add(parts[t].abs_g[k].s);
      ag[k].add(parts[t].abs_g[k].c);
    }
  }
  double v = tot.value();
  /* the number of events, or with weights their sum W */
  double nw = w ? ws.value() : (double)n;
  if (wsum_out) *wsum_out = nw;
  if (m.extended) {
    /* Poisson term for the expected count nu: nu - N ln nu (N -> W with
     * weights); nu is one parameter or the sum of the root's yields, and
     * d/d nu_j = 1 - N / nu for each of them */
    double nu = total_yield(m, th);
    v += nu - nw * std::log(nu);
    if (m.yield_param >= 0) {
      g[m.yield_param].add(1.0 - nw / nu);
    } else {
      const orc_node& ys = m.node[extended_sum(m)];
      for (int k = 0; k < ys.n_param; ++k) g[ys.param[k]].add(1.0 - nw / nu);
    }
  }
  *nll = v;
  if (grad)
    for (int k = 0; k < np; ++k) grad[k] = m.par_free[k] ? g[k].value() : 0.0;
  if (bhhh) {
    for (int j = 0; j < np; ++j)
      for (int k = j; k < np; ++k) {
        Neumaier o;
        for (int t = 0; t < T; ++t) {
          o.add(parts[t].outer[(size_t)j * np + k].s);
          o.add(parts[t].outer[(size_t)j * np + k].c);
        }
        double b = o.value();
        if (m.extended && is_yield(m, j) && is_yield(m, k)) {
          double nu = total_yield(m, th);
          b += (double)n / (nu * nu);
        }
        if (!m.par_free[j] || !m.par_free[k]) b = 0.0;
        bhhh[(size_t)j * np + k] = b;
        bhhh[(size_t)k * np + j] = b;
      }
  }
  if (stats) {
    stats[0] = al.value();
    for (int k = 0; k < np; ++k) stats[1 + k] = ag[k].value();
  }
  return ORC_OK;
}

/* Gradient descent with step halving, see oracle.h. */
/* w (may be NULL): event weights; the step is then scaled by 1/W, W their
 * sum (the weighted analogue of the mean NLL). */
/* accept_ulps: the largest computed increase of the NLL, in units of
 * DBL_EPSILON * |NLL_acc|, still taken as no increase (4 by default, 0 for
 * the literal rule). */
int gd_fit_one(const orc_model& m, const double* const* cols, int64_t n, double* theta,
               int n_steps, double eta, int threads, double* nll_out, double* grad_out,
               double* eta_out, double* trace, const double* w = nullptr,
               double accept_ulps = 4.0) {
  const int np = m.n_param;
  std::vector<double> acc(theta, theta + np), prop(theta, theta + np), g_acc(np, 0.0),
      g(np, 0.0);
  double f_acc = kInf;
  double inv_n = 1.0 / (double)std::max<int64_t>(n, 1);
  if (w) {
    Neumaier W;
    for (int64_t i = 0; i < n; ++i) W.add(w[i]);
    inv_n = W.value() > 0.0 ? 1.0 / W.value() : 1.0;
  }
  int last = ORC_OK;
  for (int s = 0; s < n_steps; ++s) {
    double f;
    int st = nll_one(m, cols, n, prop.data(), threads, &f, g.data(), nullptr, nullptr, w);
    if (trace) {
      trace[s * (np + 1)] = f;
      for (int k = 0; k < np; ++k) trace[s * (np + 1) + 1 + k] = prop[k];
    }
    /* a computed increase within the evaluation's own rounding (a few ulps
     * of the NLL) is not an increase of the function */
    bool ok = (st == ORC_OK) && std::isfinite(f) &&
              (f <= f_acc || f - f_acc <= accept_ulps * DBL_EPSILON * std::fabs(f_acc));
    if (st == ORC_E_DOMAIN) return st;
    if (ok) {
      acc = prop;
      f_acc = f;
      g_acc = g;
      last = ORC_OK;
    } else {
      eta *= 0.5;
      if (!std::isfinite(f_acc)) last = st;
    }
    for (int k = 0; k < np; ++k)
      prop[k] = m.par_free[k] ? acc[k] - eta * g_acc[k] * inv_n : acc[k];
  }
  for (int k = 0; k < np; ++k) theta[k] = acc[k];
  *nll_out = f_acc;
  if (grad_out)
    for (int k = 0; k < np; ++k) grad_out[k] = g_acc[k];
  if (eta_out) *eta_out = eta;
  return std::isfinite(f_acc) ? ORC_OK : (last != ORC_OK ? last : ORC_E_PDF);
}

/* Solve (B + lambda D) d = -g over the free parameters by Cholesky, D the
 * diagonal of B floored at 1e-12 of its largest entry; d = 0 for fixed
 * parameters.  Returns false if the damped matrix is not positive definite
 * (a pivot <= 0 or not finite). */
bool damped_solve(const orc_model& m, const double* B, const double* g, double lambda, double* d) {
  const int np = m.n_param;
  int idx[ORC_MAX_PAR];
  int nf = 0;
  double dmax = 0.0;
  for (int k = 0; k < np; ++k)
    if (m.par_free[k]) {
      idx[nf++] = k;
      dmax = std::max(dmax, B[(size_t)k * np + k]);
    }
  for (int k = 0; k < np; ++k) d[k] = 0.0;
  if (nf == 0) return true;
  std::vector<double> A((size_t)nf * nf), L((size_t)nf * nf, 0.0), y(nf);
  for (int a = 0; a < nf; ++a)
    for (int b = 0; b < nf; ++b) {
      double v = B[(size_t)idx[a] * np + idx[b]];
      if (a == b) v += lambda * std::max(v, 1e-12 * dmax);
      A[(size_t)a * nf + b] = v;
    }
  for (int a = 0; a < nf; ++a) {
    for (int b = 0; b <= a; ++b) {
      double s = A[(size_t)a * nf + b];
      for (int c = 0; c < b; ++c) s -= L[(size_t)a * nf + c] * L[(size_t)b * nf + c];
      if (a == b) {
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        L[(size_t)a * nf + a] = std::sqrt(s);
      } else {
        L[(size_t)a * nf + b] = s / L[(size_t)b * nf + b];
      }
    }
  }
  for (int a = 0; a < nf; ++a) { /* L y = -g */
    double s = -g[idx[a]];
    for (int c = 0; c < a; ++c) s -= L[(size_t)a * nf + c] * y[c];
    y[a] = s / L[(size_t)a * nf + a];
  }
  for (int a = nf - 1; a >= 0; --a) { /* L^T d = y */
    double s = y[a];
    for (int c = a + 1; c < nf; ++c) s -= L[(size_t)c * nf + a] * d[idx[c]];
    d[idx[a]] = s / L[(size_t)a * nf + a];
  }
  return true;
}

/* Damped BHHH (Levenberg-Marquardt on the outer-product matrix), see
 * oracle.h. */
int bhhh_fit_one(const orc_model& m, const double* const* cols, int64_t n, double* theta,
                 int n_steps, double lambda, int threads, double* nll_out, double* grad_out,
                 double* lambda_out, double* trace) {
  const int np = m.n_param;
  std::vector<double> acc(theta, theta + np), prop(theta, theta + np), g_acc(np, 0.0), g(np, 0.0),
      B_acc((size_t)np * np, 0.0), B((size_t)np * np, 0.0), d(np, 0.0);
  double f_acc = kInf;
  int last = ORC_OK;
  for (int s = 0; s < n_steps; ++s) {
    double f;
    int st = nll_one(m, cols, n, prop.data(), threads, &f, g.data(), nullptr, B.data());
    if (trace) {
      trace[s * (np + 1)] = f;
      for (int k = 0; k < np; ++k) trace[s * (np + 1) + 1 + k] = prop[k];
    }
    if (st == ORC_E_DOMAIN) return st;
    bool ok = (st == ORC_OK) && std::isfinite(f) && f <= f_acc + 4.0 * DBL_EPSILON * std::fabs(f_acc);
    if (ok) {
      acc = prop;
      f_acc = f;
      g_acc = g;
      B_acc = B;
      lambda = std::max(lambda * 0.1, 1e-12);
      last = ORC_OK;
    } else {
      lambda *= 10.0;
      if (!std::isfinite(f_acc)) last = st;
    }
    /* the next proposal; a damped matrix that is not positive definite is
       retried with ten times the damping, at most 8 times */
    bool solved = false;
    for (int tries = 0; tries < 8 && !solved; ++tries) {
      solved = damped_solve(m, B_acc.data(), g_acc.data(), lambda, d.data());
      if (!solved) lambda *= 10.0;
    }
    for (int k = 0; k < np; ++k) prop[k] = solved && m.par_free[k] ? acc[k] + d[k] : acc[k];
  }
  for (int k = 0; k < np; ++k) theta[k] = acc[k];
  *nll_out = f_acc;
  if (grad_out)
    for (int k = 0; k < np; ++k) grad_out[k] = g_acc[k];
  if (lambda_out) *lambda_out = lambda;
  return std::isfinite(f_acc) ? ORC_OK : (last != ORC_OK ? last : ORC_E_PDF);
}

template <class F>
void parallel_sets(int n_sets, int threads, F&& fn) {
  int T = std::max(1, std::min(threads, n_sets));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      int s = next.fetch_add(1);
      if (s >= n_sets) return;
      fn(s);
    }
  };
  if (T == 1) {
    work();
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) pool.emplace_back(work);
  for (auto& t : pool) t.join();
}

bool data_args_ok(const orc_model* m, const double* const* cols) {
  if (!m || !cols) return false;
  for (int o = 0; o < m->n_obs; ++o)
    if (!cols[o]) return false;
  return true;
}

}  // namespace

/* ------------------------------------------------------------------ */
/* C interface                                                          */
/* ------------------------------------------------------------------ */
extern "C" {

int orc_check_model(const orc_model* m) { return m ? check_model(*m) : ORC_E_ARG; }

int orc_leaf_norm(const orc_model* m, int32_t node, const double* theta, double* Z, double* dZ) {
  if (!m || !theta || !Z || !dZ) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  if (node < 0 || node >= m->n_node || !is_leaf(m->node[node].kind)) return ORC_E_ARG;
  st = check_params(*m, theta);
  if (st != ORC_OK) return st;
  double d[ORC_NODE_PAR];
  const orc_node& nd = m->node[node];
  leaf_norm_local(*m, nd, theta, Z, d);
  for (int k = 0; k < m->n_param; ++k) dZ[k] = 0.0;
  for (int k = 0; k < nd.n_param; ++k) dZ[nd.param[k]] += d[k];
  return ORC_OK;
}

int orc_log_density(const orc_model* m, const double* x, const double* theta, double* logp,
                    double* dlogp) {
  if (!m || !x || !theta || !logp) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  Prepared pr;
  st = prepare(*m, theta, pr);
  if (st != ORC_OK) return st;
  for (int o = 0; o < m->n_obs; ++o)
    if (!(x[o] >= m->lo[o] && x[o] <= m->hi[o])) return ORC_E_DOMAIN;
  double dv[ORC_MAX_PAR];
  double p = node_value(pr, m->root, x, dlogp ? dv : nullptr);
  if (!(p > 0.0) || !std::isfinite(p)) {
    *logp = -kInf;
    return ORC_E_PDF;
  }
  *logp = std::log(p);
  if (dlogp)
    for (int k = 0; k < m->n_param; ++k) dlogp[k] = dv[k] / p;
  return ORC_OK;
}

int orc_nll(const orc_model* m, const double* const* cols, int64_t n, const double* theta,
            int32_t threads, double* nll, double* grad, double* stats) {
  if (!data_args_ok(m, cols) || !theta || !nll || n < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return nll_one(*m, cols, n, theta, threads, nll, grad, stats);
}

int orc_nll_weighted(const orc_model* m, const double* const* cols, const double* w, int64_t n,
                     const double* theta, int32_t threads, double* nll, double* grad, double* stats,
                     double* wsum) {
  if (!data_args_ok(m, cols) || !w || !theta || !nll || n < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return nll_one(*m, cols, n, theta, threads, nll, grad, stats, nullptr, w, wsum);
}

int orc_gd_fit_weighted(const orc_model* m, const double* const* cols, const double* w, int64_t n,
                        double* theta, int32_t n_steps, double eta, int32_t threads, double* nll,
                        double* grad, double* eta_out, double* trace) {
  if (!data_args_ok(m, cols) || !w || !theta || !nll || n < 0 || n_steps < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return gd_fit_one(*m, cols, n, theta, n_steps, eta, threads, nll, grad, eta_out, trace, w);
}

int orc_nll_batched(const orc_model* m, const double* const* cols, const int64_t* offsets,
                    int32_t n_sets, const double* theta, int32_t threads, double* nll,
                    double* grad, int32_t* status) {
  if (!data_args_ok(m, cols) || !offsets || !theta || !nll || n_sets < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  for (int s = 0; s < n_sets; ++s)
    if (offsets[s + 1] < offsets[s]) return ORC_E_ARG;
  const int np = m->n_param;
  parallel_sets(n_sets, threads, [&](int s) {
    const double* c[ORC_MAX_OBS];
    for (int o = 0; o < m->n_obs; ++o) c[o] = cols[o] + offsets[s];
    int r = nll_one(*m, c, offsets[s + 1] - offsets[s], theta + (size_t)s * np, 1, &nll[s],
                    grad ? grad + (size_t)s * np : nullptr, nullptr);
    if (status) status[s] = r;
  });
  return ORC_OK;
}

int orc_nll_bhhh(const orc_model* m, const double* const* cols, int64_t n, const double* theta,
                 int32_t threads, double* nll, double* grad, double* bhhh) {
  if (!data_args_ok(m, cols) || !theta || !nll || !bhhh || n < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return nll_one(*m, cols, n, theta, threads, nll, grad, nullptr, bhhh);
}

int orc_bhhh_fit(const orc_model* m, const double* const* cols, int64_t n, double* theta,
                 int32_t n_steps, double lambda, int32_t threads, double* nll, double* grad,
                 double* lambda_out, double* trace) {
  if (!data_args_ok(m, cols) || !theta || !nll || n < 0 || n_steps < 0 || !(lambda > 0.0)) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return bhhh_fit_one(*m, cols, n, theta, n_steps, lambda, threads, nll, grad, lambda_out, trace);
}

int orc_gd_fit(const orc_model* m, const double* const* cols, int64_t n, double* theta,
               int32_t n_steps, double eta, int32_t threads, double* nll, double* grad,
               double* eta_out, double* trace) {
  if (!data_args_ok(m, cols) || !theta || !nll || n < 0 || n_steps < 0) return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return gd_fit_one(*m, cols, n, theta, n_steps, eta, threads, nll, grad, eta_out, trace);
}

int orc_gd_fit_accept(const orc_model* m, const double* const* cols, int64_t n, double* theta,
                      int32_t n_steps, double eta, double accept_ulps, int32_t threads,
                      double* nll, double* grad, double* eta_out, double* trace) {
  if (!data_args_ok(m, cols) || !theta || !nll || n < 0 || n_steps < 0 || !(accept_ulps >= 0.0))
    return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  return gd_fit_one(*m, cols, n, theta, n_steps, eta, threads, nll, grad, eta_out, trace, nullptr,
                    accept_ulps);
}

int orc_gd_fit_batched(const orc_model* m, const double* const* cols, const int64_t* offsets,
                       int32_t n_sets, double* theta, int32_t n_steps, double eta,
                       int32_t threads, double* nll, double* grad, int32_t* status) {
  if (!data_args_ok(m, cols) || !offsets || !theta || !nll || n_sets < 0 || n_steps < 0)
    return ORC_E_ARG;
  int st = check_model(*m);
  if (st != ORC_OK) return st;
  const int np = m->n_param;
  parallel_sets(n_sets, threads, [&](int s) {
    const double* c[ORC_MAX_OBS];
    for (int o = 0; o < m->n_obs; ++o) c[o] = cols[o] + offsets[s];
    int r = gd_fit_one(*m, c, offsets[s + 1] - offsets[s], theta + (size_t)s * np, n_steps,
                       eta, 1, &nll[s], grad ? grad + (size_t)s * np : nullptr, nullptr,
                       nullptr);
    if (status) status[s] = r;
  });
  return ORC_OK;
}

/* log K_nu(z) by the oracle's own integral (for its pins). */
int orc_log_bessel_k(double nu, double z, double* out) {
  if (!out || !(z > 0.0)) return ORC_E_ARG;
  *out = log_bessel_k(nu, z);
  return ORC_OK;
}

int orc_gl_rule(int32_t n, double* x, double* w) {
  if (n < 1 || n > 4096 || !x || !w) return ORC_E_ARG;
  Rule r = make_rule(n);
  for (int i = 0; i < n; ++i) {
    x[i] = r.x[i];
    w[i] = r.w[i];
  }
  return ORC_OK;
}

}  // extern "C"
