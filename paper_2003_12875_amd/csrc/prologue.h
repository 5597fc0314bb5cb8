// prologue.h -- per-parameter-point constants, computed once per evaluation
// (the caching of parameter-only branches of Sec. 5.1) by one thread block.
//
//  * parameter range checks (Sec. 3, "Checking parameters");
//  * per leaf: event constants, gradient scales, Z and dZ/dtheta, either in
//    closed form ("Analytic Integrals", Sec. 3) or by a 256-point
//    Gauss-Legendre rule, one node per thread, on panels where the integrand
//    is analytic (the Crystal Ball split at its junction; the ARGUS
//    endpoint removed by m = m0 - s^2) or on one panel;
//  * per term: log of its weight (product of sum coefficients) minus the
//    log normalisations of its leaves, and d log w_k / d theta.
#pragma once

#include <hip/hip_runtime.h>

#include "leaves.h"
#include "model.h"
#include "plan.h"

namespace nllmi {

constexpr int kGLNodes = 256;  // Gauss-Legendre nodes per panel, one per thread

// sum over the first kGLNodes threads (4 waves) of NV values per thread, in
// a fixed order (deterministic); the other threads of a larger block only
// take part in the barriers.
template <int NV>
__device__ inline void block_sum_small(double (&v)[NV], double* lds /* >= 4*NV */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_xor(v[j], off, 64);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0 && wave < kGLNodes / 64) {
#pragma unroll
    for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = ((lds[j] + lds[NV + j]) + lds[2 * NV + j]) + lds[3 * NV + j];
  __syncthreads();
}

// Gauss-Legendre contribution of this thread's node to Z and dZ of a leaf.
template <class Leaf>
__device__ inline void gl_node(const double* p, int norm, double lo, double hi, const double* glx,
                               const double* glw, double (&v)[Leaf::NP + 1]) {
  const int i = threadIdx.x;
  double dg[kMaxLeafParams];
#pragma unroll
  for (int j = 0; j <= Leaf::NP; ++j) v[j] = 0.0;
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
  } else {
    panel(lo, hi);
  }
}

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

// Fills *pt (LDS or global) for the parameter vector theta.  pl and theta
// are the block's LDS copies (stage_plan, stage_theta, or values written by
// the calling threads); all threads of the block must call it; on return
// *pt is complete and visible to the block.
template <class M, int NT = kBlock>
__device__ __forceinline__ void compute_pertheta(const Plan& pl, const double* theta, const double* __restrict__ glx,
                                 const double* __restrict__ glw, PerTheta* pt, double* lds) {
  static_assert(NT >= kGLNodes && NT % 64 == 0, "at least one thread per quadrature node");
  const int tid = threadIdx.x;
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  // parallel zero fill of the term-weight derivatives
  for (int i = tid; i < kMaxTerms * kMaxParams; i += NT) (&pt->dlogw[0][0])[i] = 0.0;
  __syncthreads();
  // parameter range checks (Sec. 3): one thread per parameter, per sum
  if (tid < pl.n_param) {
    const double v = theta[tid];
    if (!(v >= pl.par_lo[tid] && v <= pl.par_hi[tid])) atomicOr(&s_bad, 1);  // NaN fails too
  } else if (tid >= 64 && tid < 64 + pl.n_sum) {
    const int q = tid - 64;
    double f = 0.0;
    bool ok = true;
    for (int j = 0; j < pl.sum_nchild[q] - 1; ++j) {
      const double v = theta[pl.sum_param[q][j]];
      ok = ok && v >= 0.0 && v <= 1.0;
      f += v;
    }
    if (!ok || !(f <= 1.0)) atomicOr(&s_bad, 1);
  } else if (tid == 128 && pl.extended && !(theta[pl.yield_param] > 0.0)) {
    atomicOr(&s_bad, 1);
  }

  // (1) numerically normalised leaves: every thread evaluates one
  // Gauss-Legendre node, one leaf after the other
  static_for<M::L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    using Leaf = typename M::template S<l>::Leaf;
    if (pl.leaf_norm[l] != kNormAnalytic) {
      double p[Leaf::NP];
#pragma unroll
      for (int j = 0; j < Leaf::NP; ++j) p[j] = theta[pl.leaf_param[l][j]];
      const double lo = pl.lo[pl.leaf_obs[l]], hi = pl.hi[pl.leaf_obs[l]];
      const bool ok = Leaf::valid(p) && !(Leaf::kKind == kArgus && !(p[0] > lo));
      double v[Leaf::NP + 1];
      if (ok && tid < kGLNodes) {
        gl_node<Leaf>(p, pl.leaf_norm[l], lo, hi, glx, glw, v);
      } else {
#pragma unroll
        for (int j = 0; j <= Leaf::NP; ++j) v[j] = 0.0;
      }
      block_sum_small<Leaf::NP + 1>(v, lds);
      if (tid == 0) {
        pt->logz[l] = v[0];  // Z for now
#pragma unroll
        for (int j = 0; j < Leaf::NP; ++j) pt->dlogz[l][j] = v[j + 1];  // dZ for now
      }
    }
  });
  __syncthreads();

  // (2) per-leaf constants and closed-form integrals, leaf l on wave l % 4
  static_for<M::L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    using Leaf = typename M::template S<l>::Leaf;
    if (tid == 64 * (l % 4) + l / 4) {
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
      if (ok) Leaf::setup(p, lo, hi, analytic, s);
      if (!analytic) {
        s.Z = pt->logz[l];
        for (int j = 0; j < Leaf::NP; ++j) s.dZ[j] = pt->dlogz[l][j];
      }
      if constexpr (Leaf::kKind == kArgus) {
        if (!pl.par_free[pl.leaf_param[l][0]]) s.ec[3] = 0.0;  // m0 not differentiated
      }
      if (!ok || !(s.Z > 0.0) || !__builtin_isfinite(s.Z)) atomicOr(&s_bad, 1);
      for (int j = 0; j < kLeafConsts; ++j) pt->ec[l][j] = s.ec[j];
      const double iz = 1.0 / s.Z;
      // the FP32 pass evaluates the leaf on x - x0: its log-density is off
      // by the constant kappa, absorbed here into the normalisation
      pt->logz[l] = M::PREC == 1 ? log(s.Z) - s.kappa : log(s.Z);
      for (int j = 0; j < kMaxLeafParams; ++j) {
        pt->fscale[l][j] = s.fscale[j];
        pt->dlogz[l][j] = j < Leaf::NP ? s.dZ[j] * iz : 0.0;
        pt->phioff[l][j] = M::PREC == 1 ? s.phioff[j] : 0.0;
      }
    }
  });
  __syncthreads();

  // (3) term constants, one lane per term: log w_k - sum_{non-root l in S_k}
  // log Z_l and d log w_k / d theta over the fraction parameters of every sum
  // on the path.  Coefficients are floored at 1e-200 so that a fraction at
  // exactly 0 or 1 keeps a finite log and a finite d/df (the floored term
  // then carries a weight of 1e-200, i.e. nothing, in the likelihood).
  const int k = tid;
  if (k < kMaxTerms) {
    double lw = 0.0;
    if (k < M::K) {
      for (int r = 0; r < pl.term_nref[k]; ++r) {
        const int q = pl.term_ref_sum[k][r], j = pl.term_ref_child[k][r];
        const int nc = pl.sum_nchild[q];
        double f = 0.0;
        for (int i = 0; i < nc - 1; ++i) f += theta[pl.sum_param[q][i]];
        const double c = (j < nc - 1) ? theta[pl.sum_param[q][j]] : 1.0 - f;
        const double cf = fmax(c, 1e-200);
        lw += log(cf);
        if (j < nc - 1) {
          pt->dlogw[k][pl.sum_param[q][j]] += 1.0 / cf;
        } else {
          for (int i = 0; i < nc - 1; ++i) pt->dlogw[k][pl.sum_param[q][i]] -= 1.0 / cf;
        }
      }
      const int mask = pl.term_mask[k];
#pragma unroll
      for (int l = 0; l < M::L; ++l)
        if (!M::ROOTs[l] && ((mask >> l) & 1)) lw -= pt->logz[l];
    }
    pt->ck[k] = lw;
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
