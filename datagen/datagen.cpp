/*
 * datagen.cpp -- seeded synthetic event generator shared by the tests and
 * the benchmark (input generation only: it evaluates no likelihood,
 * normalisation or gradient).
 *
 * Randomness: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), a counter-based generator, so the
 * value drawn for event i does not depend on threading.  Event i of a
 * stream uses counters (i, j, 0, 0), j = 0, 1, ... as it consumes blocks of
 * four 64-bit words; the key is (seed, stream).
 *
 * Sampling follows the default of the paper (Sec. 3, "Generating Samples"):
 * accept/reject under a constant envelope, except where an exact inverse
 * transform is trivial (exponential) or a textbook method exists
 * (Box-Muller for the Gaussian, rejected outside the range).
 */
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <map>
#include <cstdint>
#include <thread>
#include <vector>

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  __uint128_t p = (__uint128_t)a * (__uint128_t)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds: multipliers and Weyl key increments as
 * published by Salmon et al. */
void philox4x64_10(const uint64_t in[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Per-event stream of 64-bit words. */
struct EventRng {
  uint64_t key[2];
  uint64_t index;
  uint64_t block = 0;
  uint64_t buf[4];
  int pos = 4;
  EventRng(uint64_t seed, uint64_t stream, uint64_t i) : index(i) {
    key[0] = seed;
    key[1] = stream;
  }
  uint64_t next() {
    if (pos == 4) {
      uint64_t ctr[4] = {index, block++, 0, 0};
      philox4x64_10(ctr, key, buf);
      pos = 0;
    }
    return buf[pos++];
  }
  /* uniform on [0, 1) from the top 53 bits */
  double u01() { return (double)(next() >> 11) * 0x1.0p-53; }
  /* uniform on (0, 1] */
  double u01_open0() { return (double)((next() >> 11) + 1) * 0x1.0p-53; }
};

}  // namespace

extern "C" {

typedef struct dg_node {
  int32_t kind; /* 1 gauss, 2 exp, 3 cheb, 4 cb, 5 argus, 6 sum, 7 prod, 8 johnson, 9 chi2, 10 hypatia */
  int32_t obs;
  int32_t n_param;
  double p[12]; /* parameter VALUES (truth) */
  int32_t n_child;
  int32_t child[8];
} dg_node;

typedef struct dg_model {
  int32_t n_obs;
  double lo[4], hi[4];
  int32_t n_node;
  dg_node node[16];
  int32_t root;
} dg_model;

}  // extern "C"

namespace {

constexpr int kMaxTries = 1 << 24;

double sample_gauss(EventRng& r, double mu, double s, double lo, double hi) {
  for (int t = 0; t < kMaxTries; ++t) {
    double u1 = r.u01_open0(), u2 = r.u01();
    double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2);
    double x = mu + s * z;
    if (x >= lo && x <= hi) return x;
  }
  return std::nan("");
}

/* Johnson S_U by its defining transformation: n standard normal,
 * x = mu + lambda sinh((n - gamma)/delta), kept when inside [lo, hi]. */
double sample_johnson(EventRng& r, double mu, double la, double ga, double de, double lo, double hi) {
  for (int t = 0; t < kMaxTries; ++t) {
    double u1 = r.u01_open0(), u2 = r.u01();
    double n = std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2);
    double x = mu + la * std::sinh((n - ga) / de);
    if (x >= lo && x <= hi) return x;
  }
  return std::nan("");
}

/* standard normal by Box-Muller (one of the pair) */
double normal01(EventRng& r) {
  double u1 = r.u01_open0(), u2 = r.u01();
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(kTwoPi * u2);
}

/* Gamma(k, 1) by Marsaglia and Tsang's squeeze method (k >= 1); for k < 1
 * Gamma(k + 1) U^(1/k). */
double sample_gamma(EventRng& r, double k) {
  if (k < 1.0) return sample_gamma(r, k + 1.0) * std::pow(r.u01_open0(), 1.0 / k);
  double d = k - 1.0 / 3.0, c = 1.0 / std::sqrt(9.0 * d);
  for (int t = 0; t < kMaxTries; ++t) {
    double n = normal01(r);
    double v = 1.0 + c * n;
    if (v <= 0.0) continue;
    v = v * v * v;
    double u = r.u01_open0();
    if (std::log(u) < 0.5 * n * n + d - d * v + d * std::log(v)) return d * v;
  }
  return std::nan("");
}

/* chi-square with nu degrees of freedom = 2 Gamma(nu/2, 1), kept when in [lo, hi] */
double sample_chi2(EventRng& r, double nu, double lo, double hi) {
  for (int t = 0; t < kMaxTries; ++t) {
    double x = 2.0 * sample_gamma(r, 0.5 * nu);
    if (x >= lo && x <= hi) return x;
  }
  return std::nan("");
}

double sample_exp(EventRng& r, double c, double lo, double hi) {
  double u = r.u01();
  double w = hi - lo;
  double x;
  if (std::fabs(c * w) < 1e-12)
    x = lo + u * w;
  else
    x = lo + std::log1p(u * std::expm1(c * w)) / c;
  return std::min(hi, std::max(lo, x));
}

double shape_cheb(const dg_node& nd, double lo, double hi, double x) {
  double y = (2.0 * x - lo - hi) / (hi - lo);
  double a = 1.0, b = y, g = 1.0;
  for (int k = 0; k < nd.n_param; ++k) {
    g += nd.p[k] * b;
    double nx = 2.0 * y * b - a;
    a = b;
    b = nx;
  }
  return g;
}

double shape_cb(const dg_node& nd, double x) {
  double m0 = nd.p[0], s = nd.p[1], al = nd.p[2], n = nd.p[3];
  double t = (x - m0) / s;
  if (t > -al) return std::exp(-0.5 * t * t);
  double A = std::pow(n / al, n) * std::exp(-0.5 * al * al);
  return A * std::pow(n / al - al - t, -n);
}

double shape_argus(const dg_node& nd, double x) {
  double m0 = nd.p[0], c = nd.p[1];
  if (x >= m0) return 0.0;
  double u = (m0 - x) * (m0 + x) / (m0 * m0);
  return x * std::sqrt(u) * std::exp(c * u);
}

/* accept/reject with a uniform proposal on [lo, hi] and envelope M */
template <class F>
double accept_reject(EventRng& r, double lo, double hi, double M, F&& shape) {
  for (int t = 0; t < kMaxTries; ++t) {
    double x = lo + (hi - lo) * r.u01();
    if (x > hi) x = hi;
    double y = M * r.u01();
    if (y < shape(x)) return x;
  }
  return std::nan("");
}


/* Hypatia2 for sampling: its log-density on 16384 cells of the range,
 * events drawn exactly from the piecewise log-linear interpolant of it (a
 * cell by its mass, then the inverse distribution function of the
 * exponential segment inside the cell).  The density: with d = x - mu,
 * nu = lambda - 1/2, delta^2 = sigma^2 zeta K_lambda(zeta)/K_{lambda+1}(zeta),
 * alpha = zeta/delta, the core r^nu e^{beta d} K_nu(alpha r), r^2 = d^2 +
 * delta^2, between -a_l sigma and a_r sigma, continued on each side by a
 * power law with the core's value and slope there.  K_nu from its integral
 * over exp(-z cosh t) cosh(nu t) by the trapezoidal rule. */
double dg_log_k(double nu, double z) {
  const double h = std::min(1.0 / 16.0, 0.25 / std::sqrt(z));
  double sum = 0.5;
  for (int j = 1; j < 100000; ++j) {
    const double t = j * h;
    const double term = std::exp(-z * (std::cosh(t) - 1.0)) * std::cosh(nu * t);
    sum += term;
    if (term < 1e-17 * sum && t > 1.0) break;
  }
  return std::log(h * sum) - z;
}

struct HypTable {
  std::vector<double> cum;  /* cumulative mass at the cell ends */
  std::vector<double> lg;   /* log-density at the cell edges */
  double lo, h;
};

const HypTable& hyp_table(const dg_node& nd, double lo, double hi) {
  static std::mutex mu;
  static std::map<std::vector<double>, HypTable> cache;
  std::vector<double> key(nd.p, nd.p + 9);
  key.push_back(lo);
  key.push_back(hi);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const double m0 = nd.p[0], sg = nd.p[1], la = nd.p[2], ze = nd.p[3], be = nd.p[4];
  const double al = nd.p[5], nl = nd.p[6], ar = nd.p[7], nr = nd.p[8];
  const double nu = la - 0.5;
  const double d2 = sg * sg * ze * std::exp(dg_log_k(la, ze) - dg_log_k(la + 1.0, ze));
  const double alpha = ze / std::sqrt(d2);
  auto core = [&](double d) {
    const double r2 = d * d + d2;
    return 0.5 * nu * std::log(r2) + be * d + dg_log_k(nu, alpha * std::sqrt(r2));
  };
  const double dl = -al * sg, dh = ar * sg, e = 1e-6 * sg;
  const double Gl = core(dl), sl = (core(dl + e) - core(dl - e)) / (2 * e);
  const double Gh = core(dh), sh = (core(dh + e) - core(dh - e)) / (2 * e);
  auto logg = [&](double d) {
    if (d < dl) return Gl - nl * std::log(1.0 + sl * (dl - d) / nl);
    if (d > dh) return Gh - nr * std::log(1.0 - sh * (d - dh) / nr);
    return core(d);
  };
  const int cells = 16384;
  HypTable t;
  t.lo = lo;
  t.h = (hi - lo) / cells;
  t.lg.resize(cells + 1);
  double top = -1e300;
  for (int i = 0; i <= cells; ++i) {
    t.lg[i] = logg(lo + i * t.h - m0);
    top = std::max(top, t.lg[i]);
  }
  t.cum.resize(cells);
  double acc = 0.0;
  for (int i = 0; i < cells; ++i) {
    const double a = t.lg[i] - top, c = t.lg[i + 1] - t.lg[i];
    const double w = std::fabs(c) > 1e-9 ? std::expm1(c) / c : 1.0 + 0.5 * c;
    acc += t.h * std::exp(a) * w;
    t.cum[i] = acc;
  }
  return cache.emplace(key, std::move(t)).first->second;
}

double sample_hypatia(EventRng& r, const dg_node& nd, double lo, double hi) {
  const HypTable& t = hyp_table(nd, lo, hi);
  const double u = r.u01() * t.cum.back();
  const int i = (int)(std::upper_bound(t.cum.begin(), t.cum.end(), u) - t.cum.begin());
  if (i >= (int)t.cum.size()) return hi;
  const double prev = i > 0 ? t.cum[i - 1] : 0.0;
  const double v = (u - prev) / (t.cum[i] - prev);  /* position of u within the cell's mass */
  const double c = t.lg[i + 1] - t.lg[i];
  const double s = std::fabs(c) > 1e-9 ? std::log1p(v * std::expm1(c)) / c : v;
  return std::min(hi, std::max(lo, t.lo + (i + s) * t.h));
}

void sample_node(const dg_model& m, int i, EventRng& r, double* x) {
  const dg_node& nd = m.node[i];
  double lo = (nd.obs >= 0) ? m.lo[nd.obs] : 0.0, hi = (nd.obs >= 0) ? m.hi[nd.obs] : 0.0;
  switch (nd.kind) {
    case 1: x[nd.obs] = sample_gauss(r, nd.p[0], nd.p[1], lo, hi); return;
    case 2: x[nd.obs] = sample_exp(r, nd.p[0], lo, hi); return;
    case 3: {
      double M = 1.0;
      for (int k = 0; k < nd.n_param; ++k) M += std::fabs(nd.p[k]);
      x[nd.obs] = accept_reject(r, lo, hi, M, [&](double v) { return shape_cheb(nd, lo, hi, v); });
      return;
    }
    case 4: /* the shape never exceeds 1 (its value at t = 0) */
      x[nd.obs] = accept_reject(r, lo, hi, 1.0, [&](double v) { return shape_cb(nd, v); });
      return;
    case 5: {
      double m0 = nd.p[0], c = nd.p[1];
      double top = std::min(hi, m0);
      /* sqrt(u) e^{cu} increases up to u* = -1/(2c) (c < 0): bound it on
       * [0, u(lo)] and bound m by top */
      double ulo = (m0 - lo) * (m0 + lo) / (m0 * m0);
      double us = (c < 0.0) ? std::min(ulo, -0.5 / c) : ulo;
      double M = 1.0000001 * top * std::sqrt(us) * std::exp(c * us);
      if (c >= 0.0) M = 1.0000001 * top * std::sqrt(ulo) * std::exp(c * ulo);
      x[nd.obs] = accept_reject(r, lo, top, M, [&](double v) { return shape_argus(nd, v); });
      return;
    }
    case 6: {
      double u = r.u01(), acc = 0.0;
      for (int k = 0; k < nd.n_child - 1; ++k) {
        acc += nd.p[k];
        if (u < acc) {
          sample_node(m, nd.child[k], r, x);
          return;
        }
      }
      sample_node(m, nd.child[nd.n_child - 1], r, x);
      return;
    }
    case 7:
      for (int k = 0; k < nd.n_child; ++k) sample_node(m, nd.child[k], r, x);
      return;
    case 8:
      x[nd.obs] = sample_johnson(r, nd.p[0], nd.p[1], nd.p[2], nd.p[3], lo, hi);
      return;
    case 9:
      x[nd.obs] = sample_chi2(r, nd.p[0], lo, hi);
      return;
    case 10:
      x[nd.obs] = sample_hypatia(r, nd, lo, hi);
      return;
  }
}

template <class F>
void parallel_for(int64_t n, int threads, F&& fn) {
  int T = std::max(1, threads);
  if (n < 65536) T = 1;
  if (T == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) {
    int64_t b = n * t / T, e = n * (t + 1) / T;
    pool.emplace_back([&fn, b, e]() { fn(b, e); });
  }
  for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

void dg_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  philox4x64_10(ctr, key, out);
}

/* n uniforms on [0,1): value k is the first draw of "event" k of the stream. */
void dg_uniforms(uint64_t seed, uint64_t stream, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    EventRng r(seed, stream, (uint64_t)i);
    out[i] = r.u01();
  }
}

/* Events [0, n) of stream `stream` into cols[obs][0..n).  Returns the number
 * of events for which sampling failed (NaN written). */
int64_t dg_generate(const dg_model* m, uint64_t seed, uint64_t stream, int64_t n,
                    double* const* cols, int32_t threads) {
  std::atomic<int64_t> bad{0};
  parallel_for(n, threads, [&](int64_t b, int64_t e) {
    double x[4];
    int64_t nb = 0;
    for (int64_t i = b; i < e; ++i) {
      EventRng r(seed, stream, (uint64_t)i);
      sample_node(*m, m->root, r, x);
      for (int o = 0; o < m->n_obs; ++o) {
        cols[o][i] = x[o];
        if (std::isnan(x[o])) ++nb;
      }
    }
    bad += nb;
  });
  return bad.load();
}

/* Many datasets at once: set s (model models[s], stream stream_base + s)
 * fills events [offsets[s], offsets[s+1]) of the concatenated columns. */
int64_t dg_generate_sets(const dg_model* models, int32_t n_sets, const int64_t* offsets,
                         uint64_t seed, uint64_t stream_base, double* const* cols,
                         int32_t threads) {
  std::atomic<int64_t> bad{0};
  std::atomic<int> next{0};
  int T = std::max(1, threads);
  auto work = [&]() {
    double x[4];
    for (;;) {
      int s = next.fetch_add(1);
      if (s >= n_sets) return;
      const dg_model& m = models[s];
      int64_t nb = 0;
      for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) {
        EventRng r(seed, stream_base + (uint64_t)s, (uint64_t)(i - offsets[s]));
        sample_node(m, m.root, r, x);
        for (int o = 0; o < m.n_obs; ++o) {
          cols[o][i] = x[o];
          if (std::isnan(x[o])) ++nb;
        }
      }
      bad += nb;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 0; t < T; ++t) pool.emplace_back(work);
  for (auto& th : pool) th.join();
  return bad.load();
}

}  // extern "C"
