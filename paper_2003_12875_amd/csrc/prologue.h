// prologue.h -- per-parameter-point constants, computed once per evaluation
// (the caching of parameter-only branches of Sec. 5.1) by one thread block.
//
//  * parameter range checks (Sec. 3, "Checking parameters");
//  * per leaf: event constants, gradient scales, Z and dZ/dtheta, either in
//    closed form ("Analytic Integrals", Sec. 3) or by a 256-point
//    Gauss-Legendre rule, one node per thread, on panels where the integrand
//    is analytic (the Crystal Ball split at its junction; the ARGUS
//    endpoint removed by m = m0 - s^2, the chi-square's at 0 by x = s^2)
//    or on one panel;
//  * per term: log of its weight (product of sum coefficients) minus the
//    log normalisations of its leaves, and d log w_k / d theta.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "leaves.h"
#include "model.h"
#include "plan.h"

namespace nllmi {

constexpr int kGLNodes = 256;  // Gauss-Legendre nodes per panel, one per thread

// sum over the first W waves of NV values per thread (W = 4: the first
// kGLNodes threads), in a fixed order (deterministic); the other threads of
// a larger block only take part in the barriers.
template <int NV, int W = kGLNodes / 64>
__device__ inline void block_sum_small(double (&v)[NV], double* lds /* >= 4*NV */) {
  static_assert(W == 2 || W == 4, "waves in the sum");
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_xor(v[j], off, 64);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0 && wave < W) {
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if constexpr (W == 4) {
      v[j] = ((lds[j] + lds[NV + j]) + lds[2 * NV + j]) + lds[3 * NV + j];
    } else {
      v[j] = lds[j] + lds[NV + j];
    }
  }
  __syncthreads();
}

// Lanes of the per-point set-up (compute_pertheta, phase 2): leaf l's
// group, the parameter range checks (two runs of 16 lanes), the sum checks
// and the term weights, disjoint for up to kMaxLeaves leaves.  256 threads
// or more: leaf l at 64 (l % 4) + 32 (l / 4), checks at 144 and 176, sums at
// 80, weights at 208; 128 threads (models with at most 4 leaves): leaf l at
// 32 l, checks at 16 and 48, sums at 80, weights at 112.
template <int NT>
struct PtLanes {
  static constexpr int kMaxLeaves = NT >= 256 ? 8 : 4;
  static constexpr int leaf(int l) { return NT >= 256 ? 64 * (l % 4) + 32 * (l / 4) : 32 * l; }
  static constexpr int kParA = NT >= 256 ? 144 : 16;
  static constexpr int kParB = NT >= 256 ? 176 : 48;
  static constexpr int kSum = 80;
  static constexpr int kTerm = NT >= 256 ? 208 : 112;
};

// Gauss-Legendre contribution of node i (of every panel) to Z and dZ of a
// leaf, added to v.
template <class Leaf>
__device__ inline void gl_node(const double* p, int norm, double lo, double hi, const double* glx,
                               const double* glw, int i, double (&v)[Leaf::NP + 1]) {
  double dg[kMaxLeafParams];
  auto panel = [&](double a, double b) {
    const double h = 0.5 * (b - a), c = 0.5 * (a + b);
    const double w = h * glw[i];
    const double g = Leaf::shape(p, lo, hi, fma(h, glx[i], c), dg);
    v[0] += w * g;
#pragma unroll
    for (int j = 0; j < Leaf::NP; ++j) v[j + 1] += w * dg[j];
  };
  if (norm == kNormGLSingle) {
    panel(lo, hi);
    return;
  }
  if constexpr (Leaf::kKind == kCB) {
    const double mj = p[0] - p[2] * p[1];
    if (mj > lo && mj < hi) {
      panel(lo, mj);
      panel(mj, hi);
    } else {
      panel(lo, hi);
    }
  } else if constexpr (Leaf::kKind == kArgus) {
    const double m0 = p[0];
    const double sa = sqrt(m0 - fmin(hi, m0)), sb = sqrt(fmax(m0 - lo, 0.0));
    const double h = 0.5 * (sb - sa), c = 0.5 * (sa + sb);
    const double w = h * glw[i];
    const double g = ArgusLeaf::shape_subst(p, fma(h, glx[i], c), dg);
    v[0] += w * g;
    v[1] += w * dg[0];
    v[2] += w * dg[1];
  } else if constexpr (Leaf::kKind == kChi2) {
    if (lo == 0.0) {  // x = s^2 removes the x^{nu/2-1} endpoint behaviour
      const double sb = sqrt(hi), h = 0.5 * sb;
      const double w = h * glw[i];
      const double g = Chi2Leaf::shape_subst(p, fma(h, glx[i], h), dg);
      v[0] += w * g;
      v[1] += w * dg[0];
    } else {
      panel(lo, hi);
    }
  } else {
    panel(lo, hi);
  }
}

// Expected event count of an extended model: one parameter, or the sum of
// the yields of the root's sum of yields.
__device__ inline double expected_count(const Plan& pl, const double* theta) {
  if (pl.ext_sum < 0) return theta[pl.yield_param];
  double nu = 0.0;
  for (int j = 0; j < pl.sum_nchild[pl.ext_sum]; ++j) nu += theta[pl.sum_param[pl.ext_sum][j]];
  return nu;
}
// parameter q enters the expected event count
__device__ inline bool is_count_param(const Plan& pl, int q) {
  if (pl.ext_sum < 0) return q == pl.yield_param;
  bool in = false;
  for (int j = 0; j < pl.sum_nchild[pl.ext_sum]; ++j) in = in || pl.sum_param[pl.ext_sum][j] == q;
  return in;
}

// The words of PerTheta that a model of shape M reads once the prologue
// has written them: its leaves' rows (event constants, feature scales,
// d log Z, log Z; the FP32 pass's feature offsets), its terms' constants
// and d log w rows over the parameters, and the status word.  Kernels pass
// only these between launches (a one-leaf model's are ~0.5 KB of the
// 4.5 KB block), so per-set constant traffic follows the model's size.
template <class M>
struct PtWords {
  static constexpr int L = M::L, K = M::K;
  static constexpr int kEc = (int)(__builtin_offsetof(PerTheta, ec) / 8);
  static constexpr int kFs = (int)(__builtin_offsetof(PerTheta, fscale) / 8);
  static constexpr int kDz = (int)(__builtin_offsetof(PerTheta, dlogz) / 8);
  static constexpr int kLz = (int)(__builtin_offsetof(PerTheta, logz) / 8);
  static constexpr int kCk = (int)(__builtin_offsetof(PerTheta, ck) / 8);
  static constexpr int kCr = (int)(__builtin_offsetof(PerTheta, croot) / 8);
  static constexpr int kDw = (int)(__builtin_offsetof(PerTheta, dlogw) / 8);
  static constexpr int kPo = (int)(__builtin_offsetof(PerTheta, phioff) / 8);
  static constexpr int kBad = (int)(__builtin_offsetof(PerTheta, bad) / 8);
  static constexpr int kFixed = L * (kLeafConsts + 2 * kMaxLeafParams + 1) + K + 1 +
                                (M::PREC == 1 ? L * kMaxLeafParams : 0) + 1;
  static constexpr int kMax = kFixed + K * kMaxParams;
  static_assert(sizeof(PerTheta) % 8 == 0 && __builtin_offsetof(PerTheta, bad) % 8 == 0, "8-byte words");
  __device__ static int count(int P) { return kFixed + K * P; }
  // offset (in 8-byte words) of the i-th word, i < count(P)
  __device__ static int word(int i, int P) {
    if (i < L * kLeafConsts) return kEc + i;
    i -= L * kLeafConsts;
    if (i < L * kMaxLeafParams) return kFs + i;
    i -= L * kMaxLeafParams;
    if (i < L * kMaxLeafParams) return kDz + i;
    i -= L * kMaxLeafParams;
    if (i < L) return kLz + i;
    i -= L;
    if (i < K) return kCk + i;
    i -= K;
    if (i == 0) return kCr;
    i -= 1;
    if (i == 0) return kBad;
    i -= 1;
    if constexpr (M::PREC == 1) {
      if (i < L * kMaxLeafParams) return kPo + i;
      i -= L * kMaxLeafParams;
    }
    return kDw + (i / P) * kMaxParams + i % P;  // d log w rows, P words each
  }
};

// Copy the words M reads from src to dst with NT threads (no barrier).
template <class M, int NT>
__device__ inline void copy_pertheta(PerTheta* dst, const PerTheta* src, int P) {
  using W = PtWords<M>;
  const double* s = reinterpret_cast<const double*>(src);
  double* d = reinterpret_cast<double*>(dst);
  for (int i = threadIdx.x; i < W::count(P); i += NT) {
    const int o = W::word(i, P);
    d[o] = s[o];
  }
}

// The same copy through registers: load() issues this thread's loads (so
// that they can overlap other work), store() writes them.
template <class M, int NT>
struct PtRegs {
  static constexpr int N = (PtWords<M>::kMax + NT - 1) / NT;
  double v[N];
  // every lane loads (lanes past the words read word 0, which store()
  // drops), with neither a branch nor a select after the load, so that the
  // waits that follow count these loads exactly
  __device__ void load(const PerTheta* src, int P) {
    const double* s = reinterpret_cast<const double*>(src);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int i = threadIdx.x + j * NT;
      v[j] = s[i < PtWords<M>::count(P) ? PtWords<M>::word(i, P) : 0];
    }
  }
  __device__ void store(PerTheta* dst, int P) const {
    double* d = reinterpret_cast<double*>(dst);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int i = threadIdx.x + j * NT;
      if (i < PtWords<M>::count(P)) d[PtWords<M>::word(i, P)] = v[j];
    }
  }
};

// Copies of the plan and of a parameter vector into LDS, so that the
// prologue's lane-varying and chained look-ups (parameter ranges, leaf
// parameter indices, sum coefficients) cost one parallel load instead of a
// chain of dependent ones.  No barrier: compute_pertheta starts with one.
// Callers issue these before their first event-tile loads (loads complete
// in order).
template <int NT>
__device__ inline void stage_plan(const Plan& src, Plan* dst) {
  static_assert(sizeof(Plan) % 8 == 0, "plan copied as 8-byte words");
  const uint2* s = reinterpret_cast<const uint2*>(&src);
  uint2* d = reinterpret_cast<uint2*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(Plan) / 8); i += NT) d[i] = s[i];
}
__device__ inline void stage_theta(const double* __restrict__ theta_g, int n_param, double* dst) {
  if ((int)threadIdx.x < n_param) dst[threadIdx.x] = theta_g[threadIdx.x];
}

// The plan's words in registers, NT threads each holding up to N of them:
// a kernel start that issues all its loads (plan, parameters, constants,
// records, the first event tiles) before it writes any of them to LDS
// waits for each only when it stores it, instead of one round trip per
// staged copy.  Every lane loads (lanes past the plan read word 0).
template <int NT>
struct PlanRegs {
  static constexpr int W = (int)(sizeof(Plan) / 8);
  static constexpr int N = (W + NT - 1) / NT;
  uint2 w[N];
  __device__ void load(const Plan& src) {
    const uint2* s = reinterpret_cast<const uint2*>(&src);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int i = (int)threadIdx.x + j * NT;
      w[j] = s[i < W ? i : 0];
    }
  }
  __device__ void store(Plan* dst) const {
    uint2* d = reinterpret_cast<uint2*>(dst);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int i = (int)threadIdx.x + j * NT;
      if (i < W) d[i] = w[j];
    }
  }
};

// Fills *pt for the parameter vector theta.  pl and theta are the block's
// LDS copies (stage_plan, stage_theta, or values written by the calling
// threads); *pt should be LDS (its phases read back what other threads
// wrote).  All threads of the block must call it; on return *pt is
// complete and visible to the block.  Phases:
//   (0) the per-point tables of a leaf that has them (into aux, LDS: all
//       threads, with barriers);
//   (1) leaves normalised numerically: one Gauss-Legendre node per thread,
//       two with 128 threads (skipped, with its barrier, when every leaf has
//       a closed form);
//   (2) in parallel: leaf l's constants and closed-form integrals on its
//       lane group (lanes cooperating where the leaf provides it), the
//       parameter range checks (Sec. 3) and the term weights log w_k,
//       d log w_k on lanes that hold no leaf (PtLanes);
//   (3) term constants log w_k - sum log Z over the term's non-root leaves.
template <class M, int NT = kBlock>
__device__ __forceinline__ void compute_pertheta(const Plan& pl, const double* theta, const double* __restrict__ glx,
                                 const double* __restrict__ glw, PerTheta* pt, double* lds,
                                 double* aux = nullptr) {
  // quadrature nodes: one per thread (256 threads or more) or two (128)
  static_assert(NT % 64 == 0 && (NT >= kGLNodes || 2 * NT == kGLNodes), "one or two quadrature nodes per thread");
  constexpr int W = (NT < kGLNodes ? NT : kGLNodes) / 64;  // waves in the node sums
  using LN = PtLanes<NT>;
  static_assert(M::L <= LN::kMaxLeaves, "leaf lane groups");
  static_assert(!M::AUX || NT >= kGLNodes, "per-point tables: 256 threads or more");
  static_assert(kMaxParams <= 32 && kMaxSums + 1 <= 16 && kMaxTerms <= 16, "check and weight lanes");
  const int tid = threadIdx.x;
  __shared__ int s_bad;
  __shared__ double s_lw[kMaxTerms];
  if (tid == 0) s_bad = 0;
  for (int i = tid; i < kMaxTerms * kMaxParams; i += NT) (&pt->dlogw[0][0])[i] = 0.0;
  __syncthreads();

  // (0)
  if constexpr (M::AUX) {
    static_for<M::L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      using Leaf = typename M::template S<l>::Leaf;
      if constexpr (Leaf::kAux) {
        double p[Leaf::NP];
#pragma unroll
        for (int j = 0; j < Leaf::NP; ++j) p[j] = theta[pl.leaf_param[l][j]];
        Leaf::template setup_aux<NT>(p, pl.lo[pl.leaf_obs[l]], pl.hi[pl.leaf_obs[l]], aux);
      }
    });
  }

  // (1)
  bool any_gl = false;
#pragma unroll
  for (int l = 0; l < M::L; ++l) any_gl = any_gl || pl.leaf_norm[l] != kNormAnalytic;
  if (any_gl) {
    static_for<M::L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      using Leaf = typename M::template S<l>::Leaf;
      if (pl.leaf_norm[l] != kNormAnalytic) {
        double p[Leaf::NP];
#pragma unroll
        for (int j = 0; j < Leaf::NP; ++j) p[j] = theta[pl.leaf_param[l][j]];
        const double lo = pl.lo[pl.leaf_obs[l]], hi = pl.hi[pl.leaf_obs[l]];
        if constexpr (Leaf::kOwnNorm) {
          // composite rule on 1, 2, 4, ... panels until two successive
          // levels agree to 1e-13 of the integral of |g| and 1e-11 of those
          // of |dg/dp_k| (a level that resolves the density is exact to
          // rounding, so agreement means the finer one is); no agreement
          // within kJitMaxPanels panels leaves Z = NaN, an invalid density
          constexpr int NV = Leaf::NP + 1;
          double zp[NV], zc[NV], ab[NV];
          auto level = [&](int n_pan, double (&z)[NV]) {
#pragma unroll
            for (int j = 0; j < NV; ++j) z[j] = ab[j] = 0.0;
            for (int i = tid; i < kGLNodes; i += NT) {
              double zi[NV], ai[NV];
              Leaf::norm_level(p, lo, hi, n_pan, glx, glw, i, zi, ai);
#pragma unroll
              for (int j = 0; j < NV; ++j) {
                z[j] += zi[j];
                ab[j] += ai[j];
              }
            }
            block_sum_small<NV, W>(z, lds);
            block_sum_small<NV, W>(ab, lds);
          };
          level(1, zp);
          bool conv = false;
          for (int n_pan = 2; n_pan <= kJitMaxPanels && !conv; n_pan *= 2) {
            level(n_pan, zc);
            conv = __builtin_isfinite(zc[0]) && fabs(zc[0] - zp[0]) <= 1e-13 * ab[0];
#pragma unroll
            for (int j = 1; j < NV; ++j) conv = conv && fabs(zc[j] - zp[j]) <= 1e-11 * ab[j];
#pragma unroll
            for (int j = 0; j < NV; ++j) zp[j] = zc[j];
          }
          if (tid == 0) {
            pt->logz[l] = conv ? zp[0] : __builtin_nan("");  // Z for now
#pragma unroll
            for (int j = 0; j < Leaf::NP; ++j) pt->dlogz[l][j] = zp[j + 1];  // dZ for now
          }
        } else {
          const bool ok = Leaf::valid(p) && !(Leaf::kKind == kArgus && !(p[0] > lo));
          double v[Leaf::NP + 1];
#pragma unroll
          for (int j = 0; j <= Leaf::NP; ++j) v[j] = 0.0;
          if (ok) {
            if constexpr (Leaf::kAux) {
              if (tid < kGLNodes) Leaf::gl_norm(aux, lo, hi, glx, glw, v);
            } else {
              for (int i = tid; i < kGLNodes; i += NT) gl_node<Leaf>(p, pl.leaf_norm[l], lo, hi, glx, glw, i, v);
            }
          }
          block_sum_small<Leaf::NP + 1, W>(v, lds);
          if (tid == 0) {
            pt->logz[l] = v[0];  // Z for now
#pragma unroll
            for (int j = 0; j < Leaf::NP; ++j) pt->dlogz[l][j] = v[j + 1];  // dZ for now
          }
        }
      }
    });
    __syncthreads();
  }

  // (2a) leaf l: lanes [LN::leaf(l), LN::leaf(l) + Leaf::kSetupLanes)
  static_for<M::L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    using Leaf = typename M::template S<l>::Leaf;
    constexpr int owner = LN::leaf(l);
    static_assert(Leaf::kSetupLanes >= 1 && Leaf::kSetupLanes <= 16, "setup lanes");
    if (tid >= owner && tid < owner + Leaf::kSetupLanes) {
      const int lane = tid - owner;
      double p[Leaf::NP];
#pragma unroll
      for (int j = 0; j < Leaf::NP; ++j) p[j] = theta[pl.leaf_param[l][j]];
      const double lo = pl.lo[pl.leaf_obs[l]], hi = pl.hi[pl.leaf_obs[l]];
      const bool analytic = pl.leaf_norm[l] == kNormAnalytic;
      const bool ok = Leaf::valid(p) && !(Leaf::kKind == kArgus && !(p[0] > lo));
      LeafSetup s;
      for (int j = 0; j < kLeafConsts; ++j) s.ec[j] = 0.0;
      for (int j = 0; j < kMaxLeafParams; ++j) {
        s.fscale[j] = 0.0;
        s.dZ[j] = 0.0;
        s.phioff[j] = 0.0;
      }
      s.Z = 0.0;
      s.kappa = 0.0;
      if constexpr (Leaf::kAux) {  // constants in the tables; features are d/d parameter
#pragma unroll
        for (int j = 0; j < Leaf::NP; ++j) s.fscale[j] = 1.0;
        if (!Leaf::aux_ok(aux)) atomicOr(&s_bad, 1);
      } else if (ok) {
        if constexpr (Leaf::kSetupLanes > 1) {
          Leaf::setup_coop(p, lo, hi, analytic, s, lane);
        } else {
          Leaf::setup(p, lo, hi, analytic, s);
        }
      }
      if (lane == 0) {
        if (!analytic) {
          s.Z = pt->logz[l];
          for (int j = 0; j < Leaf::NP; ++j) s.dZ[j] = pt->dlogz[l][j];
        }
        if constexpr (Leaf::kKind == kArgus) {
          if (!pl.par_free[pl.leaf_param[l][0]]) s.ec[3] = 0.0;  // m0 not differentiated
        }
        // a parameter outside a leaf's domain: bit 0; a formula leaf whose
        // normalisation is not positive and finite (or did not converge):
        // bit 1, an invalid density rather than an invalid parameter
        if (!ok || !(s.Z > 0.0) || !__builtin_isfinite(s.Z)) atomicOr(&s_bad, Leaf::kOwnNorm ? 2 : 1);
        for (int j = 0; j < kLeafConsts; ++j) pt->ec[l][j] = s.ec[j];
        const double iz = 1.0 / s.Z;
        // the FP32 pass evaluates the leaf on x - x0: its log-density is off
        // by the constant kappa, absorbed here into the normalisation
        const double lz = log_pos(s.Z);  // Z > 0 finite unless flagged just above
        pt->logz[l] = M::PREC == 1 ? lz - s.kappa : lz;
        for (int j = 0; j < kMaxLeafParams; ++j) {
          pt->fscale[l][j] = s.fscale[j];
          pt->dlogz[l][j] = j < Leaf::NP ? s.dZ[j] * iz : 0.0;
          pt->phioff[l][j] = M::PREC == 1 ? s.phioff[j] : 0.0;
        }
      }
    }
  });

  // (2b) checks (Sec. 3) on lanes no leaf uses (PtLanes): parameter ranges,
  // one lane per parameter; sum fractions in [0, 1] with a sum <= 1 (or
  // yields >= 0 with a positive finite total), one lane per sum node, and a
  // positive expected count
  if ((tid >= LN::kParA && tid < LN::kParA + 16) || (tid >= LN::kParB && tid < LN::kParB + 16)) {
    const int q = tid < LN::kParA + 16 ? tid - LN::kParA : tid - LN::kParB + 16;
    if (q < pl.n_param) {
      const double v = theta[q];
      if (!(v >= pl.par_lo[q] && v <= pl.par_hi[q])) atomicOr(&s_bad, 1);  // NaN fails too
    }
  } else if (tid >= LN::kSum && tid < LN::kSum + kMaxSums) {
    const int qs = tid - LN::kSum;
    if (qs < pl.n_sum) {
      double f = 0.0;
      bool ok = true;
      if (pl.sum_yields[qs]) {
        for (int j = 0; j < pl.sum_nchild[qs]; ++j) {
          const double v = theta[pl.sum_param[qs][j]];
          ok = ok && v >= 0.0;
          f += v;
        }
        ok = ok && f > 0.0 && __builtin_isfinite(f);
      } else {
        for (int j = 0; j < pl.sum_nchild[qs] - 1; ++j) {
          const double v = theta[pl.sum_param[qs][j]];
          ok = ok && v >= 0.0 && v <= 1.0;
          f += v;
        }
        ok = ok && f <= 1.0;
      }
      if (!ok) atomicOr(&s_bad, 1);
    }
  } else if (tid == LN::kSum + kMaxSums) {
    if (pl.extended && !(expected_count(pl, theta) > 0.0)) atomicOr(&s_bad, 1);
  }

  // (2c) term weights, one lane per term (PtLanes): log w_k and
  // d log w_k / d theta over the coefficient parameters of every sum on the
  // path: a fraction f_j (the last child 1 - sum f), or a yield's share
  // nu_j / S with S = sum nu (d log / d nu_i = [i = j] / nu_j - 1 / S).
  // Coefficients (yields) are floored at 1e-200 so that one at exactly 0
  // (or a last fraction at 0) keeps a finite log and derivative (the
  // floored term then carries a weight of 1e-200, i.e. nothing, in the
  // likelihood).
  if (tid >= LN::kTerm && tid < LN::kTerm + M::K) {
    const int k = tid - LN::kTerm;
    double lw = 0.0;
    for (int r = 0; r < pl.term_nref[k]; ++r) {
      const int q = pl.term_ref_sum[k][r], j = pl.term_ref_child[k][r];
      const int nc = pl.sum_nchild[q];
      if (pl.sum_yields[q]) {
        double S = 0.0;
        for (int i = 0; i < nc; ++i) S += theta[pl.sum_param[q][i]];
        const double cf = fmax(theta[pl.sum_param[q][j]], 1e-200);
        lw += log_pos(cf) - log_pos(S);
        pt->dlogw[k][pl.sum_param[q][j]] += 1.0 / cf;
        const double is = 1.0 / S;
        for (int i = 0; i < nc; ++i) pt->dlogw[k][pl.sum_param[q][i]] -= is;
        continue;
      }
      double f = 0.0;
      for (int i = 0; i < nc - 1; ++i) f += theta[pl.sum_param[q][i]];
      const double c = (j < nc - 1) ? theta[pl.sum_param[q][j]] : 1.0 - f;
      const double cf = fmax(c, 1e-200);
      lw += log_pos(cf);
      if (j < nc - 1) {
        pt->dlogw[k][pl.sum_param[q][j]] += 1.0 / cf;
      } else {
        for (int i = 0; i < nc - 1; ++i) pt->dlogw[k][pl.sum_param[q][i]] -= 1.0 / cf;
      }
    }
    s_lw[k] = lw;
  }
  __syncthreads();

  // (3) term constants: log w_k - sum_{non-root l in S_k} log Z_l
  if (tid < kMaxTerms) {
    const int k = tid;
    double ck = 0.0;
    if (k < M::K) {
      ck = s_lw[k];
      const int mask = pl.term_mask[k];
#pragma unroll
      for (int l = 0; l < M::L; ++l)
        if (!M::ROOTs[l] && ((mask >> l) & 1)) ck -= pt->logz[l];
    }
    pt->ck[k] = ck;
  } else if (tid == 64) {
    double croot = 0.0;
#pragma unroll
    for (int l = 0; l < M::L; ++l)
      if (M::ROOTs[l]) croot -= pt->logz[l];
    pt->croot = croot;
  }
  __syncthreads();
  if (tid == 0) pt->bad = s_bad;
  __syncthreads();
}

}  // namespace nllmi
