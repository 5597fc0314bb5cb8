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
// density leaves of composite models (leaves.h, JitLeaf).
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
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; const double ib = 1.0 / b.v; for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a) { return dscale(a, -a.v, -1.0); }
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a) { return a; }
template <int N> __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> __device__ inline Dual<N> operator+(double a, const Dual<N>& b) { Dual<N> r = b; r.v += a; return r; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> __device__ inline Dual<N> operator-(double a, const Dual<N>& b) { return dscale(b, a - b.v, -1.0); }
template <int N> __device__ inline Dual<N> operator*(const Dual<N>& a, double b) { return dscale(a, a.v * b, b); }
template <int N> __device__ inline Dual<N> operator*(double a, const Dual<N>& b) { return dscale(b, a * b.v, a); }
template <int N> __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return dscale(a, a.v / b, 1.0 / b); }
template <int N> __device__ inline Dual<N> operator/(double a, const Dual<N>& b) { const double v = a / b.v; return dscale(b, v, -v / b.v); }
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
// sum over the block's 256 threads, the same order on every call
__device__ inline DD block_sum(DD v, DD* lds) {
  for (int off = 32; off >= 1; off >>= 1) {
    DD o; o.hi = __shfl_xor(v.hi, off, 64); o.lo = __shfl_xor(v.lo, off, 64);
    v = dd_add(v, o);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  const DD r = dd_add(dd_add(lds[0], lds[1]), dd_add(lds[2], lds[3]));
  __syncthreads();
  return r;
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
// The gradient features g'_k / g (never the likelihood value): for normal
// g, g'_k times the hardware reciprocal refined by one Newton step
// (relative error ~2^-48); for subnormal g, whose reciprocal overflows, the
// division itself (a divergent branch only where such an event occurs).
template <int N>
__device__ inline void add_features(const Dual<N>& g, double* f) {
  if (g.v >= 2.2250738585072014e-308) {
    const double r0 = __builtin_amdgcn_rcp(g.v);
    const double r = fma(r0, fma(-g.v, r0, 1.0), r0);
    for (int k = 0; k < N; ++k) f[k] = fma(g.d[k], r, f[k]);
  } else {
    for (int k = 0; k < N; ++k) f[k] += g.d[k] / g.v;
  }
}

// the density, as given
template <class T> __device__ inline T jit_g(double x, const T* p) { return (T)(@EXPR@); }
template <> __device__ inline Dual<NP> jit_g<Dual<NP>>(double x, const Dual<NP>* p) { return dconst<NP>(0.0) + (@EXPR@); }

// Streaming pass: per block the sum of log g and of the features
// g'_k / g, and the count of events with g <= 0 or non-finite.
template <bool GRAD>
__device__ inline void stream(const JitArgs& a) {
  constexpr int NV = 1 + (GRAD ? NP : 0) + 1;
  __shared__ DD s_red[4];
  __shared__ DD s_tot[NV];
  double l = 0.0, f[NP > 0 ? NP : 1];
  double P = 1.0;  // running product of the events' g (mantissa) and its binary exponent
  int E = 0;
  for (int k = 0; k < NP; ++k) f[k] = 0.0;
  int bad = 0;
  const i64 stride = (i64)gridDim.x * NTH;
  if (GRAD) {
    Dual<NP> p[NP];
    for (int k = 0; k < NP; ++k) {
      p[k] = dconst<NP>(a.theta[k]);
      p[k].d[k] = 1.0;
    }
    for (i64 i = (i64)blockIdx.x * NTH + threadIdx.x; i < a.n; i += stride) {
      const Dual<NP> g = jit_g<Dual<NP>>(a.x[i], p);
      const bool ok = g.v > 0.0 && isfinite(g.v);
      bad += ok ? 0 : 1;
      prod_mul(P, E, ok ? g.v : 1.0);
      if (ok) add_features(g, f);
    }
  } else {
    double p[NP > 0 ? NP : 1];
    for (int k = 0; k < NP; ++k) p[k] = a.theta[k];
    for (i64 i = (i64)blockIdx.x * NTH + threadIdx.x; i < a.n; i += stride) {
      const double g = jit_g<double>(a.x[i], p);
      const bool ok = g > 0.0 && isfinite(g);
      bad += ok ? 0 : 1;
      prod_mul(P, E, ok ? g : 1.0);
    }
  }
  l = log(P) + (double)E * 0.6931471805599453;  // the thread's sum of log g, one logarithm
  DD v; v.lo = 0.0;
  v.hi = l;
  DD t = block_sum(v, s_red);
  if (threadIdx.x == 0) s_tot[0] = t;
  if (GRAD) {
    for (int k = 0; k < NP; ++k) {
      v.hi = f[k];
      t = block_sum(v, s_red);
      if (threadIdx.x == 0) s_tot[1 + k] = t;
    }
  }
  v.hi = (double)bad;
  t = block_sum(v, s_red);
  if (threadIdx.x == 0) s_tot[NV - 1] = t;
  __syncthreads();
  if (threadIdx.x < NV) ((DD*)a.partials)[(i64)blockIdx.x * NV + threadIdx.x] = s_tot[threadIdx.x];
}

// Z and dZ/dp_k (z[0], z[1 + k]) by composite 256-point Gauss-Legendre on
// n_pan equal panels of [lo, hi], thread t taking node t of every panel,
// with the integrals of |g| and |g'_k| (sc) as their error scales.  Every
// thread returns the same values.
__device__ inline void gl_panels(const JitArgs& a, int n_pan, const Dual<NP>* p, DD* s_red, double* z,
                                 double* sc) {
  const int t = threadIdx.x;
  const double H = (a.hi - a.lo) / n_pan, h = 0.5 * H;
  const double w = h * a.glw[t], xt = a.glx[t];
  DD acc[1 + NP];
  double ab[1 + NP];
  for (int k = 0; k <= NP; ++k) {
    acc[k].hi = acc[k].lo = 0.0;
    ab[k] = 0.0;
  }
  for (int j = 0; j < n_pan; ++j) {
    const double x = j + 1 == n_pan ? fma(h, xt, a.hi - h) : fma(h, xt, fma((double)j, H, a.lo + h));
    const Dual<NP> g = jit_g<Dual<NP>>(x, p);
    acc[0] = dd_add1(acc[0], w * g.v);
    ab[0] += w * fabs(g.v);
    for (int k = 0; k < NP; ++k) {
      acc[1 + k] = dd_add1(acc[1 + k], w * g.d[k]);
      ab[1 + k] += w * fabs(g.d[k]);
    }
  }
  for (int k = 0; k <= NP; ++k) {
    const DD r = block_sum(acc[k], s_red);
    z[k] = r.hi + r.lo;
    DD q; q.hi = ab[k]; q.lo = 0.0;
    const DD rs = block_sum(q, s_red);
    sc[k] = rs.hi + rs.lo;
  }
}

// Finishing block: Z and dZ/dp_k by composite Gauss-Legendre, doubling the
// panels (1, 2, 4, ... kMaxPanels) until the last two levels agree to
// 1e-13 of the integral of |g| and 1e-11 of that of |g'_k| (a level that
// resolves the density is exact to rounding, so agreement means the finer
// one is); no agreement at kMaxPanels panels is reported as an invalid
// density.  Then the block partials in block order, and
//   NLL = -sum log g + N log Z,  dNLL/dp_k = -sum g'_k/g + N dZ_k / Z.
#define MAX_PANELS 256
template <bool GRAD>
__device__ inline void finish(const JitArgs& a) {
  constexpr int NV = 1 + (GRAD ? NP : 0) + 1;
  __shared__ DD s_red[4];
  __shared__ double s_z[1 + NP];
  __shared__ double s_s[NV];
  __shared__ int s_bad;
  const int t = threadIdx.x;
  if (t == 0) s_bad = 0;
  __syncthreads();
  if (t < NP && !(a.theta[t] >= a.par_lo[t] && a.theta[t] <= a.par_hi[t])) s_bad = 1;  // NaN fails
  Dual<NP> p[NP];
  for (int k = 0; k < NP; ++k) {
    p[k] = dconst<NP>(a.theta[k]);
    p[k].d[k] = 1.0;
  }
  double zp[1 + NP], zc[1 + NP], sc[1 + NP];
  gl_panels(a, 1, p, s_red, zp, sc);
  bool conv = false;
  for (int n_pan = 2; n_pan <= MAX_PANELS && !conv; n_pan *= 2) {
    gl_panels(a, n_pan, p, s_red, zc, sc);
    conv = isfinite(zc[0]) && fabs(zc[0] - zp[0]) <= 1e-13 * sc[0];
    for (int k = 0; k < NP; ++k) conv = conv && fabs(zc[1 + k] - zp[1 + k]) <= 1e-11 * sc[1 + k];
    for (int k = 0; k <= NP; ++k) zp[k] = zc[k];
  }
  if (t == 0)
    for (int k = 0; k <= NP; ++k) s_z[k] = zp[k];
  DD z;
  for (int j = 0; j < NV; ++j) {
    DD acc; acc.hi = 0.0; acc.lo = 0.0;
    for (int b = t; b < a.n_blocks; b += NTH) acc = dd_add(acc, ((const DD*)a.partials)[(i64)b * NV + j]);
    z = block_sum(acc, s_red);
    if (t == 0) s_s[j] = z.hi + z.lo;
  }
  __syncthreads();
  const double Z = s_z[0], N = (double)a.n;
  int status = 0;
  if (s_bad) status = -3;
  else if (s_s[NV - 1] > 0.0 || !(Z > 0.0) || !isfinite(Z) || !conv) status = -5;
  double nll = -s_s[0] + N * log(Z);
  if (status == 0 && !isfinite(nll)) status = -5;
  if (status != 0) nll = __builtin_inf();
  if (t == 0) {
    *a.nll_out = nll;
    if (status == -3) atomicOr(a.status, 1);
    if (status == -5) atomicOr(a.status, 2);
  }
  if (GRAD && a.grad_out && t < NP) {
    const double gk = status == 0 ? -s_s[1 + t] + N * s_z[1 + t] / Z : 0.0;
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
