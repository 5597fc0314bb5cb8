// jit_source.h -- device source of the just-in-time densities (Sec. 4: PDFs
// given as formula strings and compiled at run time).  The host runtime
// (host_jit.cpp) pastes the number of parameters and the density
// expression into it and compiles it with hipRTC for the device it runs on.
//
// The expression g(x; p[0..NP-1]) is instantiated twice: with p of type
// double (the NLL alone) and of type Dual<NP> (forward-mode derivatives:
// every arithmetic operation and elementary function carries d/dp_k along),
// so that the gradient features d log g / d p_k = g'_k / g come out of the
// same streaming pass.  Normalisation: the finishing block integrates g and
// its derivatives by composite 256-point Gauss-Legendre on 1, 2, 4, ...
// equal panels (node t of every panel on thread t) until two successive
// levels agree, so that a peak narrow against the range is resolved.
// Reductions are double-double, in fixed orders.
#pragma once

namespace nllmi {

// Forward-mode dual numbers over N parameters (value and d/dp_k through
// every operation and elementary function), in the global namespace so
// that the device library's functions of double stay visible beside
// them.  Pasted into both the stand-alone density program and the
// density leaves of composite models (leaves.h, JitLeaf).  A quotient
// with a dual operand is the product with the divisor's correctly rounded
// reciprocal (within about one rounding of the quotient), so that a
// divisor fixed over the events -- a parameter -- costs one division per
// pass instead of one per event; a divisor below 2^-1024 in magnitude,
// whose reciprocal overflows, gives an infinite (or NaN) quotient.
inline const char* jit_dual_source() {
  return R"JIT(
// forward-mode dual numbers
template <int N> struct Dual { double v; double d[N]; };
template <int N> __device__ inline Dual<N> dconst(double c) { Dual<N> r; r.v = c; for (int k = 0; k < N; ++k) r.d[k] = 0.0; return r; }
template <int N> __device__ inline Dual<N> dscale(const Dual<N>& a, double v, double s) {
  Dual<N> r; r.v = v; for (int k = 0; k < N; ++k) r.d[k] = s * a.d[k]; return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; const double ib = 1.0 / b.v; r.v = a.v * ib; for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a) { return dscale(a, -a.v, -1.0); }
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a) { return a; }
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> __device__ inline Dual<N> operator+(double a, const Dual<N>& b) { Dual<N> r = b; r.v += a; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> __device__ inline Dual<N> operator-(double a, const Dual<N>& b) { return dscale(b, a - b.v, -1.0); }
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, double b) { return dscale(a, a.v * b, b); }
template <int N> __device__ inline Dual<N> operator*(double a, const Dual<N>& b) { return dscale(b, a * b.v, a); }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { const double ib = 1.0 / b; return dscale(a, a.v * ib, ib); }
template <int N> __device__ inline Dual<N> operator/(double a, const Dual<N>& b) { const double ib = 1.0 / b.v, v = a * ib; return dscale(b, v, -v * ib); }
template <int N> __device__ inline Dual<N> exp(const Dual<N>& a) { const double v = exp(a.v); return dscale(a, v, v); }
template <int N> __device__ inline Dual<N> log(const Dual<N>& a) { return dscale(a, log(a.v), 1.0 / a.v); }
template <int N> __device__ inline Dual<N> sqrt(const Dual<N>& a) { const double v = sqrt(a.v); return dscale(a, v, 0.5 / v); }
template <int N> __device__ inline Dual<N> sin(const Dual<N>& a) { return dscale(a, sin(a.v), cos(a.v)); }
template <int N> __device__ inline Dual<N> cos(const Dual<N>& a) { return dscale(a, cos(a.v), -sin(a.v)); }
template <int N> __device__ inline Dual<N> tan(const Dual<N>& a) { const double v = tan(a.v); return dscale(a, v, 1.0 + v * v); }
template <int N> __device__ inline Dual<N> atan(const Dual<N>& a) { return dscale(a, atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
template <int N> __device__ inline Dual<N> tanh(const Dual<N>& a) { const double v = tanh(a.v); return dscale(a, v, 1.0 - v * v); }
template <int N> __device__ inline Dual<N> sinh(const Dual<N>& a) { return dscale(a, sinh(a.v), cosh(a.v)); }
template <int N> __device__ inline Dual<N> cosh(const Dual<N>& a) { return dscale(a, cosh(a.v), sinh(a.v)); }
template <int N> __device__ inline Dual<N> asinh(const Dual<N>& a) { return dscale(a, asinh(a.v), 1.0 / sqrt(1.0 + a.v * a.v)); }
template <int N> __device__ inline Dual<N> erf(const Dual<N>& a) { return dscale(a, erf(a.v), 1.1283791670955126 * exp(-a.v * a.v)); }
template <int N> __device__ inline Dual<N> fabs(const Dual<N>& a) { return dscale(a, fabs(a.v), a.v < 0.0 ? -1.0 : 1.0); }
template <int N> __device__ inline Dual<N> pow(const Dual<N>& a, double b) { const double v = pow(a.v, b); return dscale(a, v, b * pow(a.v, b - 1.0)); }
template <int N> __device__ inline Dual<N> pow(double a, const Dual<N>& b) { const double v = pow(a, b.v); return dscale(b, v, v * log(a)); }
template <int N> __device__ inline Dual<N> pow(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = pow(a.v, b.v); const double la = log(a.v), ia = 1.0 / a.v;
  for (int k = 0; k < N; ++k) r.d[k] = r.v * (b.d[k] * la + b.v * a.d[k] * ia);
  return r;
}
)JIT";
}

inline const char* jit_source_template() {
  return R"JIT(
typedef long long i64;
#define NTH 256
#define MAXP 8

struct JitArgs {
  const double* x;
  i64 n;
  const double* theta;
  double* nll_out;
  double* grad_out;
  double* partials;
  int* status;
  const double* glx;
  const double* glw;
  double lo, hi;
  double par_lo[MAXP], par_hi[MAXP];
  int par_free[MAXP];
  int n_blocks;
};

struct DD { double hi, lo; };
__device__ inline DD dd_add(DD x, DD y) {
  const double s = x.hi + y.hi, bb = s - x.hi;
  const double err = (x.hi - (s - bb)) + (y.hi - bb);
  const double t = err + (x.lo + y.lo), h = s + t;
  DD r; r.hi = h; r.lo = t - (h - s); return r;
}
__device__ inline DD dd_add1(DD x, double y) {
  const double s = x.hi + y, bb = s - x.hi;
  const double err = (x.hi - (s - bb)) + (y - bb);
  const double t = err + x.lo, h = s + t;
  DD r; r.hi = h; r.lo = t - (h - s); return r;
}
// K sums (K <= 64) over the block's 256 threads, each in a fixed order.
// Within a wave, recursive halving: at lane offset o = 32, 16, ... a lane
// keeps the half of its values chosen by its lane bit o and adds the
// partner lane's copy of that half, so that after log2 K rounds (K
// rounded up to a power of two) each lane holds a partial of one value,
// indexed by its upper lane bits, at half the work of a plain butterfly
// round per round; the remaining offsets add the partner's partial of the
// same value.  Then the four waves' partials through LDS (4 K entries,
// K rounded up).  Thread t < K returns the total of value t.
constexpr int pow2_at_least(int k) { return k <= 1 ? 1 : 2 * pow2_at_least((k + 1) / 2); }
constexpr int log2_of(int k) { return k <= 1 ? 0 : 1 + log2_of(k / 2); }
__device__ inline DD dd_shfl_xor(DD v, int o) {
  DD r; r.hi = __shfl_xor(v.hi, o, 64); r.lo = __shfl_xor(v.lo, o, 64); return r;
}
template <int H>
__device__ inline void halve(DD* v, int o) {
  const bool up = (threadIdx.x & o) != 0;
  for (int j = 0; j < H; ++j) {
    const DD send = up ? v[j] : v[j + H];
    const DD keep = up ? v[j + H] : v[j];
    v[j] = dd_add(keep, dd_shfl_xor(send, o));
  }
  if constexpr (H > 1) halve<H / 2>(v, o >> 1);
}
template <int K>
__device__ inline DD block_reduce(const DD* in, DD* lds) {
  static_assert(K >= 1 && K <= 64, "1 to 64 values");
  constexpr int KP = pow2_at_least(K), LG = log2_of(KP);
  DD v[KP];
  for (int k = 0; k < KP; ++k) {
    v[k].hi = k < K ? in[k].hi : 0.0;
    v[k].lo = k < K ? in[k].lo : 0.0;
  }
  if constexpr (KP > 1) halve<KP / 2>(v, 32);
  for (int o = 32 >> LG; o >= 1; o >>= 1) v[0] = dd_add(v[0], dd_shfl_xor(v[0], o));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if ((lane & ((64 >> LG) - 1)) == 0) lds[wave * KP + (lane >> (6 - LG))] = v[0];
  __syncthreads();
  DD r; r.hi = r.lo = 0.0;
  const int k = threadIdx.x;
  if (k < K) r = dd_add(dd_add(lds[k], lds[KP + k]), dd_add(lds[2 * KP + k], lds[3 * KP + k]));
  __syncthreads();
  return r;
}
// the same, with every thread receiving all K totals in v
template <int K>
__device__ inline void block_sum(DD* v, DD* lds) {
  const DD r = block_reduce<K>(v, lds);
  if ((int)threadIdx.x < K) lds[threadIdx.x] = r;
  __syncthreads();
  for (int k = 0; k < K; ++k) v[k] = lds[k];
  __syncthreads();
}

@DUAL@

// Sum of log g over a thread's events as one logarithm: the running
// product of the g, renormalised to a mantissa in [1/2, 1) and an exponent
// after every factor.  g is split into its own mantissa and exponent first,
// so that a subnormal g is multiplied in at full precision.
__device__ inline void prod_mul(double& P, int& E, double g) {
  int eg, e;
  const double m = frexp(g, &eg);
  P = frexp(P * m, &e);
  E += e + eg;
}
// The gradient features g'_k / g (never the likelihood value), added for
// events with ok (g > 0 and finite), without a branch: g'_k s times the
// hardware reciprocal of g s refined by one Newton step (relative error
// ~2^-48), with s = 2^64 for subnormal g, whose own reciprocal overflows
// (g s is then exact and normal), else s = 1.
template <int N>
__device__ inline void add_features(const Dual<N>& g, bool ok, double* f) {
  const double s = g.v < 2.2250738585072014e-308 ? 18446744073709551616.0 : 1.0;
  const double gs = g.v * s;
  const double r0 = __builtin_amdgcn_rcp(gs);
  const double r = ok ? fma(r0, fma(-gs, r0, 1.0), r0) : 0.0;
  for (int k = 0; k < N; ++k) f[k] = fma(ok ? g.d[k] * s : 0.0, r, f[k]);
}

// the density, as given
template <class T> __device__ inline T jit_g(double x, const T* p) { return (T)(@EXPR@); }
template <> __device__ inline Dual<NP> jit_g<Dual<NP>>(double x, const Dual<NP>* p) { return dconst<NP>(0.0) + (@EXPR@); }

// The thread's events i0, i0 + S, i0 + 2S, ... (S the grid's thread
// count), JU per trip: the next trip's loads are issued before this trip's
// arithmetic, so that every wave keeps JU loads in flight.  Indices past
// the last event read event n - 1 and are not used.
#define JU 8
template <class F>
__device__ inline void for_events(const JitArgs& a, F&& ev) {
  const i64 stride = (i64)gridDim.x * NTH, i0 = (i64)blockIdx.x * NTH + threadIdx.x;
  if (i0 >= a.n) return;
  const i64 m = (a.n - 1 - i0) / stride + 1, last = a.n - 1;
  double xn[JU];
  for (int u = 0; u < JU; ++u) xn[u] = a.x[min(i0 + u * stride, last)];
  for (i64 j = 0; j < m; j += JU) {
    double xc[JU];
    for (int u = 0; u < JU; ++u) xc[u] = xn[u];
    for (int u = 0; u < JU; ++u) xn[u] = a.x[min(i0 + (j + JU + u) * stride, last)];
    if (j + JU <= m) {
      for (int u = 0; u < JU; ++u) ev(xc[u]);
    } else {
      for (int u = 0; u < JU; ++u)
        if (j + u < m) ev(xc[u]);
    }
  }
}

// Streaming pass: per block the sum of log g and of the features
// g'_k / g, and the count of events with g <= 0 or non-finite.
template <bool GRAD>
__device__ inline void stream(const JitArgs& a) {
  constexpr int NV = 1 + (GRAD ? NP : 0) + 1;
  __shared__ DD s_red[4 * pow2_at_least(NV)];
  double f[NP > 0 ? NP : 1];
  double P = 1.0;  // running product of the events' g (mantissa) and its binary exponent
  int E = 0;
  for (int k = 0; k < NP; ++k) f[k] = 0.0;
  int bad = 0;
  if (GRAD) {
    Dual<NP> p[NP];
    for (int k = 0; k < NP; ++k) {
      p[k] = dconst<NP>(a.theta[k]);
      p[k].d[k] = 1.0;
    }
    for_events(a, [&](double x) {
      const Dual<NP> g = jit_g<Dual<NP>>(x, p);
      const bool ok = g.v > 0.0 && isfinite(g.v);
      bad += ok ? 0 : 1;
      prod_mul(P, E, ok ? g.v : 1.0);
      add_features(g, ok, f);
    });
  } else {
    double p[NP > 0 ? NP : 1];
    for (int k = 0; k < NP; ++k) p[k] = a.theta[k];
    for_events(a, [&](double x) {
      const double g = jit_g<double>(x, p);
      const bool ok = g > 0.0 && isfinite(g);
      bad += ok ? 0 : 1;
      prod_mul(P, E, ok ? g : 1.0);
    });
  }
  DD v[NV];
  for (int j = 0; j < NV; ++j) v[j].lo = 0.0;
  v[0].hi = log(P) + (double)E * 0.6931471805599453;  // the thread's sum of log g, one logarithm
  if (GRAD)
    for (int k = 0; k < NP; ++k) v[1 + k].hi = f[k];
  v[NV - 1].hi = (double)bad;
  const DD t = block_reduce<NV>(v, s_red);
  if (threadIdx.x < NV) ((DD*)a.partials)[(i64)blockIdx.x * NV + threadIdx.x] = t;
}

// One level of the composite 256-point Gauss-Legendre rule on n_pan equal
// panels of [lo, hi], thread t taking node t of every panel: the thread's
// sums of w g and w g'_k (v[0], v[1 + k]) and of w |g|, w |g'_k|
// (v[1 + NP], v[2 + NP + k]: the integrals' error scales).
__device__ inline void gl_level(const JitArgs& a, int n_pan, const Dual<NP>* p, DD* v) {
  const int t = threadIdx.x;
  const double H = (a.hi - a.lo) / n_pan, h = 0.5 * H;
  const double w = h * a.glw[t], xt = a.glx[t];
  double ab[1 + NP];
  for (int k = 0; k <= NP; ++k) {
    v[k].hi = v[k].lo = 0.0;
    ab[k] = 0.0;
  }
  for (int j = 0; j < n_pan; ++j) {
    const double x = j + 1 == n_pan ? fma(h, xt, a.hi - h) : fma(h, xt, fma((double)j, H, a.lo + h));
    const Dual<NP> g = jit_g<Dual<NP>>(x, p);
    v[0] = dd_add1(v[0], w * g.v);
    ab[0] += w * fabs(g.v);
    for (int k = 0; k < NP; ++k) {
      v[1 + k] = dd_add1(v[1 + k], w * g.d[k]);
      ab[1 + k] += w * fabs(g.d[k]);
    }
  }
  for (int k = 0; k <= NP; ++k) {
    v[1 + NP + k].hi = ab[k];
    v[1 + NP + k].lo = 0.0;
  }
}

// two successive levels agree: to 1e-13 of the integral of |g| and 1e-11
// of that of |g'_k| (sc: the finer level's scales)
__device__ inline bool gl_agree(const double* zp, const double* zc, const double* sc) {
  bool conv = isfinite(zc[0]) && fabs(zc[0] - zp[0]) <= 1e-13 * sc[0];
  for (int k = 0; k < NP; ++k) conv = conv && fabs(zc[1 + k] - zp[1 + k]) <= 1e-11 * sc[1 + k];
  return conv;
}

// Finishing block: Z and dZ/dp_k by composite Gauss-Legendre, doubling the
// panels (1, 2, 4, ... MAX_PANELS) until two successive levels agree (a
// level that resolves the density is exact to rounding, so agreement
// means the finer one is); no agreement at MAX_PANELS panels is reported
// as an invalid density.  The stream's block partials are summed per
// value in block order.  Then
//   NLL = -sum log g + N log Z,  dNLL/dp_k = -sum g'_k/g + N dZ_k / Z.
// The partials' first loads are issued before the quadrature, and the
// first two levels and the partials share one block reduction (three for
// more than four parameters).
#define MAX_PANELS 256
template <bool GRAD>
__device__ inline void finish(const JitArgs& a) {
  constexpr int NV = 1 + (GRAD ? NP : 0) + 1;
  constexpr int L = 2 * (1 + NP);             // values of one quadrature level
  constexpr int Q = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);  // rounds of partials loaded ahead
  __shared__ DD s_red[4 * pow2_at_least(2 * L + NV <= 32 ? 2 * L + NV : L)];
  __shared__ int s_bad;
  const int t = threadIdx.x;
  const DD* part = (const DD*)a.partials;
  DD pr[Q][NV];
  for (int q = 0; q < Q; ++q) {
    const i64 b = min(t + q * NTH, a.n_blocks - 1);
    for (int j = 0; j < NV; ++j) pr[q][j] = part[b * NV + j];
  }
  if (t == 0) s_bad = 0;
  __syncthreads();
  if (t < NP && !(a.theta[t] >= a.par_lo[t] && a.theta[t] <= a.par_hi[t])) s_bad = 1;  // NaN fails
  Dual<NP> p[NP];
  for (int k = 0; k < NP; ++k) {
    p[k] = dconst<NP>(a.theta[k]);
    p[k].d[k] = 1.0;
  }
  DD v[2 * L + NV];
  gl_level(a, 1, p, v);
  gl_level(a, 2, p, v + L);
  DD* acc = v + 2 * L;
  for (int j = 0; j < NV; ++j) acc[j].hi = acc[j].lo = 0.0;
  for (int q = 0; q < Q; ++q)
    if (t + q * NTH < a.n_blocks)
      for (int j = 0; j < NV; ++j) acc[j] = dd_add(acc[j], pr[q][j]);
  for (int b = t + Q * NTH; b < a.n_blocks; b += NTH)
    for (int j = 0; j < NV; ++j) acc[j] = dd_add(acc[j], part[(i64)b * NV + j]);
  if constexpr (2 * L + NV <= 32) {
    block_sum<2 * L + NV>(v, s_red);
  } else {  // many parameters: three narrower reductions keep the values in registers
    block_sum<L>(v, s_red);
    block_sum<L>(v + L, s_red);
    block_sum<NV>(acc, s_red);
  }
  double zp[1 + NP], zc[1 + NP], sc[1 + NP], ss[NV];
  for (int k = 0; k <= NP; ++k) {
    zp[k] = v[k].hi + v[k].lo;
    zc[k] = v[L + k].hi + v[L + k].lo;
    sc[k] = v[L + 1 + NP + k].hi + v[L + 1 + NP + k].lo;
  }
  for (int j = 0; j < NV; ++j) ss[j] = acc[j].hi + acc[j].lo;
  bool conv = gl_agree(zp, zc, sc);
  for (int k = 0; k <= NP; ++k) zp[k] = zc[k];
  for (int n_pan = 4; n_pan <= MAX_PANELS && !conv; n_pan *= 2) {
    DD w[L];
    gl_level(a, n_pan, p, w);
    block_sum<L>(w, s_red);
    for (int k = 0; k <= NP; ++k) {
      zc[k] = w[k].hi + w[k].lo;
      sc[k] = w[1 + NP + k].hi + w[1 + NP + k].lo;
    }
    conv = gl_agree(zp, zc, sc);
    for (int k = 0; k <= NP; ++k) zp[k] = zc[k];
  }
  const double Z = zp[0], N = (double)a.n;
  int status = 0;
  if (s_bad) status = -3;
  else if (ss[NV - 1] > 0.0 || !(Z > 0.0) || !isfinite(Z) || !conv) status = -5;
  double nll = -ss[0] + N * log(Z);
  if (status == 0 && !isfinite(nll)) status = -5;
  if (status != 0) nll = __builtin_inf();
  if (t == 0) {
    *a.nll_out = nll;
    if (status == -3) atomicOr(a.status, 1);
    if (status == -5) atomicOr(a.status, 2);
  }
  if (GRAD && a.grad_out && t < NP) {
    double sk = ss[1], zk = zp[1];
    for (int k = 1; k < NP; ++k)
      if (t == k) {
        sk = ss[1 + k];
        zk = zp[1 + k];
      }
    const double gk = status == 0 ? -sk + N * zk / Z : 0.0;
    a.grad_out[t] = a.par_free[t] ? gk : 0.0;
  }
}

extern "C" __global__ __launch_bounds__(NTH) void k_jit_stream_grad(JitArgs a) { stream<true>(a); }
extern "C" __global__ __launch_bounds__(NTH) void k_jit_stream_nll(JitArgs a) { stream<false>(a); }
extern "C" __global__ __launch_bounds__(NTH) void k_jit_finish_grad(JitArgs a) { finish<true>(a); }
extern "C" __global__ __launch_bounds__(NTH) void k_jit_finish_nll(JitArgs a) { finish<false>(a); }
)JIT";
}

}  // namespace nllmi
