// histfactory.hip -- the binned template likelihood on the device: a
// persistent streaming pass over the bins (one load per template and bin,
// coalesced) and a finishing block.  HBM-bound: 8 (1 + S + H) bytes per bin.
#include <hip/hip_runtime.h>

#include "fp64.h"
#include "histfactory.h"
#include "kernels.h"
#include "reduce.h"

namespace nllmi {

// Delta templates of one histosys: up - T and T - down, once at attachment.
__global__ __launch_bounds__(kBlock) void k_hf_deltas(const double* __restrict__ nominal,
                                                      const double* __restrict__ up,
                                                      const double* __restrict__ down, int64_t n,
                                                      double* __restrict__ dup, double* __restrict__ ddn) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double t = nominal[i];
    dup[i] = up[i] - t;
    ddn[i] = t - down[i];
  }
}

// A normsys factor eta(a) and d eta / d a.  Code 0: hi^a (a >= 0), lo^-a.
// Code 1 for |a| < 1: eta = 1 + E(a) + O(a), E = c2 a^2 + c4 a^4 + c6 a^6
// and O = c1 a + c3 a^3 + c5 a^5, whose value, slope and curvature at +-1
// equal those of hi^a and lo^-a: E and O at a = 1 follow from the sums and
// differences of the six conditions, and each 3 x 3 system is solved here
// in closed form.
__device__ inline void hf_eta(double a, double lnhi, double lnlo, int code, double& eta, double& deta) {
  if (code == 1 && fabs(a) < 1.0) {
    const double hi = exp(lnhi), lo = exp(lnlo);
    const double h1 = hi * lnhi, l1 = lo * lnlo, h2 = h1 * lnhi, l2 = l1 * lnlo;
    const double E0 = 0.5 * (hi + lo) - 1.0, E1 = 0.5 * (h1 + l1), E2 = 0.5 * (h2 + l2);
    const double O0 = 0.5 * (hi - lo), O1 = 0.5 * (h1 - l1), O2 = 0.5 * (h2 - l2);
    const double c6 = 0.125 * (E2 - 5.0 * E1 + 8.0 * E0);
    const double c4 = 0.5 * (E1 - 2.0 * E0) - 2.0 * c6;
    const double c2 = E0 - c4 - c6;
    const double c5 = 0.125 * (O2 - 3.0 * O1 + 3.0 * O0);
    const double c3 = 0.5 * (O1 - O0) - 2.0 * c5;
    const double c1 = O0 - c3 - c5;
    eta = fma(a, fma(a, fma(a, fma(a, fma(a, fma(a, c6, c5), c4), c3), c2), c1), 1.0);
    deta = fma(a, fma(a, fma(a, fma(a, fma(a, 6.0 * c6, 5.0 * c5), 4.0 * c4), 3.0 * c3), 2.0 * c2), c1);
    return;
  }
  const double L = a >= 0.0 ? lnhi : -lnlo;
  eta = exp(a * L);
  deta = L * eta;
}

// A histosys delta c_u du + c_d dd (du = up - T, dd = T - down) and its
// derivative g_u du + g_d dd at a.  Code 0: a du (a >= 0), a dd.  Code 1 for
// |a| < 1: a (S + a A (15 + a^2 (3 a^2 - 10))) with S = (du + dd)/2,
// A = (du - dd)/16, i.e. c_u = a/2 + p/16, c_d = a/2 - p/16,
// p = 15 a^2 - 10 a^4 + 3 a^6.
__device__ inline void hf_histo_coef(double a, int code, double& cu, double& cd, double& gu, double& gd) {
  if (code == 1 && fabs(a) < 1.0) {
    const double a2 = a * a;
    const double p = a2 * fma(a2, fma(3.0, a2, -10.0), 15.0);
    const double dp = a * fma(a2, fma(18.0, a2, -40.0), 30.0);
    cu = fma(0.0625, p, 0.5 * a);
    cd = fma(-0.0625, p, 0.5 * a);
    gu = fma(0.0625, dp, 0.5);
    gd = fma(-0.0625, dp, 0.5);
  } else if (a >= 0.0) {
    cu = a, cd = 0.0, gu = 1.0, gd = 0.0;
  } else {
    cu = 0.0, cd = a, gu = 0.0, gd = 1.0;
  }
}

// F_s: the normfactors and normsys factors of sample s at theta (its own
// index ranges).  Shared by both kernels, so that they use the same bits.
__device__ inline double hf_factor(const HFPlan& pl, const double* theta, int s) {
  double f = 1.0;
  for (int i = pl.nf_start[s]; i < pl.nf_start[s + 1]; ++i) f *= theta[pl.nf_param[i]];
  for (int k = pl.ns_start[s]; k < pl.ns_start[s + 1]; ++k) {
    double eta, deta;
    hf_eta(theta[pl.ns_param[k]], pl.ns_lnhi[k], pl.ns_lnlo[k], pl.ns_code[k], eta, deta);
    f *= eta;
  }
  return f;
}

// lane 0's value for the whole wave (kept in scalar registers)
__device__ inline double hf_uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ inline const double* hf_uniform(const double* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return reinterpret_cast<const double*>(((uint64_t)hi << 32) | lo);
}

// The plan into LDS with one parallel copy: the set-up loops below look
// fields up by runtime indices, which from the kernel-argument segment would
// cost a dependent scalar load each.
template <int NT>
__device__ inline void hf_stage_plan(const HFPlan& src, HFPlan* dst) {
  static_assert(sizeof(HFPlan) % 8 == 0, "plan copied as 8-byte words");
  const uint2* a = reinterpret_cast<const uint2*>(&src);
  uint2* b = reinterpret_cast<uint2*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(HFPlan) / 8); i += NT) b[i] = a[i];
}

// parameter p inside its range (one thread per parameter)
__device__ inline bool hf_par_ok(const HFPlan& pl, const double* theta, int p) {
  return theta[p] >= pl.par_lo[p] && theta[p] <= pl.par_hi[p];  // NaN fails
}

// tau_b = 1/sigma_b^2 of the per-bin statistical parameters, -1 where the
// bin has none (sigma_b <= 0 or not finite), once at nll_hf_set_staterror.
__global__ __launch_bounds__(kBlock) void k_hf_tau(const double* __restrict__ sigma, int64_t n,
                                                   double* __restrict__ tau) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double s = sigma[i];
    tau[i] = (s > 0.0 && __builtin_isfinite(s)) ? 1.0 / (s * s) : -1.0;
  }
}

// STAT: the flagged samples' terms (nominal and histosys deltas) of bin b
// are summed apart, nu_b = gamma_b nu_flagged + nu_rest, their weighted sums
// take gamma_b, the bin's constraint (1/2 tau_b (gamma_b - 1)^2, or
// tau_b (gamma_b - ln gamma_b) for shapesys) joins its term, and
// d NLL / d gamma_b = w_b nu_flagged + (the constraint's derivative) is
// written per bin (0 where the bin has no parameter: gamma_b taken as 1).
// SMOOTH: every histosys reads both delta templates, adds c_u du + c_d dd
// and sums w du and w dd apart (U_h, L_h); otherwise only the template of
// alpha's side, a d, and its sum SD_h.
template <bool GRAD, bool STAT, bool SMOOTH>
__global__ __launch_bounds__(kBlock) void k_hf_stream(const HFPlan plan, const HFArgs a) {
  constexpr int NH = kHfNV / 2, NH2 = kHfNV - NH;  // two reduction passes
  constexpr int HM = SMOOTH ? kHfPolyHisto : kHfMaxHisto;  // histosys handled
  __shared__ HFPlan pl;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_F[kHfMaxSamples], s_c[kHfMaxHisto], s_cd[kHfMaxHisto];
  __shared__ int s_side[kHfMaxHisto];
  __shared__ int s_ok;
  __shared__ double red[(NH2 > NH ? NH2 : NH) * (kBlock + 1)];
  __shared__ DD tot[kHfNV];
  const int t = threadIdx.x;
  hf_stage_plan<kBlock>(plan, &pl);
  if (t < plan.n_param) s_theta[t] = a.theta[t];
  if (t == 0) s_ok = 1;
  __syncthreads();
  if (t < kHfMaxSamples) s_F[t] = t < pl.n_samples ? hf_factor(pl, s_theta, t) : 0.0;
  if (t >= 64 && t < 64 + pl.n_param && !hf_par_ok(pl, s_theta, t - 64)) s_ok = 0;
  __syncthreads();
  if (t < kHfMaxHisto) {
    const bool on = t < pl.n_histo;
    const double al = on ? s_theta[pl.histo_param[t]] : 0.0;
    const double F = on ? s_F[pl.histo_sample[t]] : 0.0;
    if constexpr (SMOOTH) {
      double cu, cd, gu, gd;
      hf_histo_coef(al, on ? pl.hs_code[t] : 0, cu, cd, gu, gd);
      s_c[t] = F * cu;
      s_cd[t] = F * cd;
    } else {
      s_c[t] = F * al;
      s_cd[t] = 0.0;
    }
    s_side[t] = al >= 0.0;
  }
  __syncthreads();
  const int S = pl.n_samples, H = pl.n_histo;
  double F[kHfMaxSamples], c[HM], c2[HM];
  const double* dp[HM];
  const double* dq[HM];
  // STAT: the flagged samples' coefficients (F_s, c_h of their histosys;
  // 0 for the others) and the rest's, uniform: nu_flagged = sum Ff_s T_s +
  // sum cf_h d_h and nu_rest = sum Fr_s T_s + sum cr_h d_h (Fr = F, cr = c
  // without STAT), so that nu = gamma_b nu_flagged + nu_rest has no
  // cancellation however small gamma_b is
  double Ff[kHfMaxSamples], cf[HM], cf2[HM], fsm[kHfMaxSamples], fhm[HM];
  double Fr[kHfMaxSamples], cr[HM], cr2[HM];
#pragma unroll
  for (int s = 0; s < kHfMaxSamples; ++s) F[s] = hf_uniform(s_F[s]);
#pragma unroll
  for (int h = 0; h < HM; ++h) {
    c[h] = hf_uniform(s_c[h]);
    c2[h] = hf_uniform(s_cd[h]);
    if constexpr (SMOOTH) {
      dp[h] = a.dup[h];  // both templates
      dq[h] = a.ddn[h];
    } else {
      dp[h] = hf_uniform(s_side[h] ? a.dup[h] : a.ddn[h]);
      dq[h] = nullptr;
    }
  }
#pragma unroll
  for (int s = 0; s < kHfMaxSamples; ++s) {
    fsm[s] = (STAT && ((pl.stat_mask >> s) & 1)) ? 1.0 : 0.0;
    Ff[s] = fsm[s] * F[s];
    Fr[s] = F[s] - Ff[s];
  }
#pragma unroll
  for (int h = 0; h < HM; ++h) {
    fhm[h] = (STAT && h < H && ((pl.stat_mask >> pl.histo_sample[h]) & 1)) ? 1.0 : 0.0;
    cf[h] = fhm[h] * c[h];
    cr[h] = c[h] - cf[h];
    cf2[h] = fhm[h] * c2[h];
    cr2[h] = c2[h] - cf2[h];
  }
  const bool poisson = STAT && pl.stat_kind == 1;
  double acc[kHfNV - 1];
#pragma unroll
  for (int j = 0; j < kHfNV - 1; ++j) acc[j] = 0.0;
  int bad = 0;
  if (s_ok) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t b = (int64_t)blockIdx.x * kBlock + t; b < a.n_bins; b += stride) {
      const double n = a.counts[b];
      double T[kHfMaxSamples], d[HM], e[HM];
#pragma unroll
      for (int s = 0; s < kHfMaxSamples; ++s) T[s] = s < S ? a.nominal[s][b] : 0.0;
#pragma unroll
      for (int h = 0; h < HM; ++h) {
        d[h] = h < H ? dp[h][b] : 0.0;
        e[h] = (SMOOTH && h < H) ? dq[h][b] : 0.0;
      }
      double nu = 0.0, nu_f = 0.0, g = 1.0, tau = 0.0;
      bool act = false;
#pragma unroll
      for (int s = 0; s < kHfMaxSamples; ++s) nu = fma(Fr[s], T[s], nu);
#pragma unroll
      for (int h = 0; h < HM; ++h) {
        nu = fma(cr[h], d[h], nu);
        if constexpr (SMOOTH) nu = fma(cr2[h], e[h], nu);
      }
      if constexpr (STAT) {
        tau = a.stat_tau[b];
        act = tau > 0.0;
        const double gb = a.gamma[b];
        g = act ? gb : 1.0;
#pragma unroll
        for (int s = 0; s < kHfMaxSamples; ++s) nu_f = fma(Ff[s], T[s], nu_f);
#pragma unroll
        for (int h = 0; h < HM; ++h) {
          nu_f = fma(cf[h], d[h], nu_f);
          if constexpr (SMOOTH) nu_f = fma(cf2[h], e[h], nu_f);
        }
        nu = fma(g, nu_f, nu);  // gamma_b nu_flagged + nu_rest
      }
      const bool pos = n > 0.0;
      bad += !(nu >= 0.0) || (pos && !(nu > 0.0));
      // n = 0: the bin contributes nu and no logarithm
      const double lnu = pos && nu > 0.0 ? log_pos(nu) : 0.0;
      acc[0] += fma(-n, lnu, nu);
      if constexpr (STAT) {
        if (act) {
          if (poisson) {
            bad += !(g > 0.0);
            acc[0] = fma(tau, g - (g > 0.0 ? log_pos(g) : 0.0), acc[0]);
          } else {
            const double dg = g - 1.0;
            acc[0] = fma(0.5 * tau * dg, dg, acc[0]);
          }
        }
      }
      if constexpr (GRAD) {
        const double w = pos ? fma(-n, rcp_full(nu), 1.0) : 1.0;
        // the flagged samples' sums take w gamma_b: w + w (gamma_b - 1) [flagged]
        const double wd = STAT ? w * (g - 1.0) : 0.0;
#pragma unroll
        for (int s = 0; s < kHfMaxSamples; ++s) acc[1 + s] = fma(fma(wd, fsm[s], w), T[s], acc[1 + s]);
#pragma unroll
        for (int h = 0; h < HM; ++h) {
          const double wh = fma(wd, fhm[h], w);
          if constexpr (SMOOTH) {
            acc[1 + kHfMaxSamples + 2 * h] = fma(wh, d[h], acc[1 + kHfMaxSamples + 2 * h]);
            acc[2 + kHfMaxSamples + 2 * h] = fma(wh, e[h], acc[2 + kHfMaxSamples + 2 * h]);
          } else {
            acc[1 + kHfMaxSamples + h] = fma(wh, d[h], acc[1 + kHfMaxSamples + h]);
          }
        }
        if constexpr (STAT) {
          if (a.grad_gamma) {
            const double dc = poisson ? tau * (1.0 - (g > 0.0 ? 1.0 / g : 0.0)) : tau * (g - 1.0);
            a.grad_gamma[b] = act ? fma(w, nu_f, dc) : 0.0;
          }
        }
      }
    }
  }
  double v0[NH], v1[NH2];
#pragma unroll
  for (int j = 0; j < NH; ++j) v0[j] = acc[j];
#pragma unroll
  for (int j = 0; j < NH2 - 1; ++j) v1[j] = acc[NH + j];
  v1[NH2 - 1] = (double)bad;
  block_sum_vals<NH, kBlock>(v0, red, tot);
  block_sum_vals<NH2, kBlock>(v1, red, tot + NH);
  if (t < kHfNV) reinterpret_cast<DD*>(a.partials)[(size_t)blockIdx.x * kHfNV + t] = tot[t];
}

// Finishing block: the partials in block order, then NLL, status and the
// gradient from the per-sample and per-histosys sums:
//   SA_s = ST_s + sum_{h on s} V_h  (= sum_b w_b (T_sb + deltas)), with
//          V_h = alpha_h SD_h, or (smooth) c_u U_h + c_d L_h
//   normfactor mu on s:  (F_s / mu) SA_s, F_s / mu formed as the product of
//                        the sample's other factors
//   normsys alpha on s:  F_s L SA_s, L = eta'(alpha) / eta(alpha) (ln hi or
//                        -ln lo for the exponential code)
//   histosys h:          F_{s_h} SD_h, or (smooth) F_{s_h} (g_u U_h + g_d L_h)
//   constrained p:       + (theta_p - m_p) / s_p^2
// Each modifier's term is formed by a thread of its own; a parameter's
// thread then adds the terms of the modifiers it drives, in modifier order.
template <bool GRAD>
__global__ __launch_bounds__(kFinishBlock) void k_hf_finish(const HFPlan plan, const HFArgs a, int n_blocks) {
  __shared__ HFPlan pl;
  __shared__ DD tot[kHfNV];
  __shared__ double s_theta[kMaxParams], s_cons[kMaxParams], s_F[kHfMaxSamples], s_SA[kHfMaxSamples];
  __shared__ double s_term[kHfSlots];
  __shared__ int s_ok;
  const int t = threadIdx.x;
  hf_stage_plan<kFinishBlock>(plan, &pl);
  if (t < plan.n_param) s_theta[t] = a.theta[t];
  if (t == 0) s_ok = 1;
  // 16 lanes per value (34 values), 16 records per lane in flight: the
  // 512 block records in two memory round trips (32 would spill at 1024
  // threads)
  RecordSum<kHfNV, kFinishBlock, 16> rs;
  rs.issue(reinterpret_cast<const DD*>(a.partials), n_blocks);
  __syncthreads();
  if (t < kHfMaxSamples) s_F[t] = t < pl.n_samples ? hf_factor(pl, s_theta, t) : 0.0;
  if (t >= 64 && t < 64 + kMaxParams) {  // range checks and constraint terms, one thread per parameter
    const int p = t - 64;
    double c = 0.0;
    if (p < pl.n_param) {
      if (!hf_par_ok(pl, s_theta, p)) s_ok = 0;
      if (pl.par_constrained[p]) {
        const double dv = s_theta[p] - pl.par_mean[p];
        c = 0.5 * dv * dv * pl.par_ivar[p];
      }
    }
    s_cons[p] = c;
  }
  rs.reduce(reinterpret_cast<const DD*>(a.partials), n_blocks, tot);  // ends with a barrier
  const auto val = [&](int j) { return tot[j].hi + tot[j].lo; };
  const bool smooth = pl.smooth_histo != 0;
  if (t < kHfMaxSamples) {
    double sa = 0.0;
    if (t < pl.n_samples) {
      sa = val(1 + t);
      for (int h = pl.hs_start[t]; h < pl.hs_start[t + 1]; ++h) {
        const double al = s_theta[pl.histo_param[h]];
        if (smooth) {
          double cu, cd, gu, gd;
          hf_histo_coef(al, pl.hs_code[h], cu, cd, gu, gd);
          sa = fma(cu, val(1 + kHfMaxSamples + 2 * h), sa);
          sa = fma(cd, val(2 + kHfMaxSamples + 2 * h), sa);
        } else {
          sa = fma(al, val(1 + kHfMaxSamples + h), sa);
        }
      }
    }
    s_SA[t] = sa;
  }
  __syncthreads();
  // one thread per modifier forms its term (slot order: normfactors,
  // normsys, histosys)
  if (t >= 64 && t < 64 + kHfSlots) {
    const int j = t - 64;
    double term = 0.0;
    if (j < kHfMaxNormfactor) {
      if (j < pl.n_normfactor) {
        const int s = pl.nf_sample[j];
        double others = 1.0;  // the sample's factors except this one
        for (int i = pl.nf_start[s]; i < pl.nf_start[s + 1]; ++i)
          if (i != j) others *= s_theta[pl.nf_param[i]];
        for (int k = pl.ns_start[s]; k < pl.ns_start[s + 1]; ++k) {
          double eta, deta;
          hf_eta(s_theta[pl.ns_param[k]], pl.ns_lnhi[k], pl.ns_lnlo[k], pl.ns_code[k], eta, deta);
          others *= eta;
        }
        term = others * s_SA[s];
      }
    } else if (j < kHfMaxNormfactor + kHfMaxNormsys) {
      const int k = j - kHfMaxNormfactor;
      if (k < pl.n_normsys) {
        const int s = pl.ns_sample[k];
        const double al = s_theta[pl.ns_param[k]];
        double L;
        if (pl.ns_code[k] == 1 && fabs(al) < 1.0) {
          double eta, deta;
          hf_eta(al, pl.ns_lnhi[k], pl.ns_lnlo[k], 1, eta, deta);
          L = deta / eta;
        } else {
          L = al >= 0.0 ? pl.ns_lnhi[k] : -pl.ns_lnlo[k];
        }
        term = s_F[s] * L * s_SA[s];
      }
    } else {
      const int h = j - kHfMaxNormfactor - kHfMaxNormsys;
      if (h < pl.n_histo) {
        if (smooth) {
          double cu, cd, gu, gd;
          hf_histo_coef(s_theta[pl.histo_param[h]], pl.hs_code[h], cu, cd, gu, gd);
          term = s_F[pl.histo_sample[h]] *
                 fma(gu, val(1 + kHfMaxSamples + 2 * h), gd * val(2 + kHfMaxSamples + 2 * h));
        } else {
          term = s_F[pl.histo_sample[h]] * val(1 + kHfMaxSamples + h);
        }
      }
    }
    s_term[j] = term;
  }
  __syncthreads();
  double nll = val(0);
#pragma unroll
  for (int p = 0; p < kMaxParams; ++p) nll += s_cons[p];
  int status = 0;
  if (!s_ok) status = -3;
  else if (val(kHfNV - 1) > 0.0 || !__builtin_isfinite(nll)) status = -5;
  if (status != 0) nll = __builtin_inf();
  if (t == 0) {
    *a.nll_out = nll;
    if (status == -3) atomicOr(a.status, (int)kStatusParam);
    if (status == -5) atomicOr(a.status, (int)kStatusPdf);
  }
  if (GRAD && a.grad_out && t < pl.n_param) {
    const int q = t;
    double g = 0.0;
    if (status == 0) {
      for (int i = pl.par_start[q]; i < pl.par_start[q + 1]; ++i) g += s_term[pl.par_slot[i]];
      if (pl.par_constrained[q]) g = fma(s_theta[q] - pl.par_mean[q], pl.par_ivar[q], g);
    }
    a.grad_out[q] = pl.par_free[q] ? g : 0.0;
  }
}

hipError_t launch_hf_deltas(const double* nominal, const double* up, const double* down, int64_t n, double* dup,
                            double* ddn, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_hf_deltas, dim3((unsigned)blocks), dim3(kBlock), 0, st, nominal, up, down, n, dup, ddn);
  return hipGetLastError();
}

hipError_t launch_hf_tau(const double* sigma, int64_t n, double* tau, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_hf_tau, dim3((unsigned)blocks), dim3(kBlock), 0, st, sigma, n, tau);
  return hipGetLastError();
}

hipError_t launch_hf_eval(const HFPlan& pl, const HFArgs& a, bool grad, int grid, hipStream_t st) {
  const bool stat = a.gamma != nullptr;
  const dim3 g(grid), b(kBlock);
  if (pl.smooth_histo) {
    if (stat) {
      if (grad) hipLaunchKernelGGL((k_hf_stream<true, true, true>), g, b, 0, st, pl, a);
      else hipLaunchKernelGGL((k_hf_stream<false, true, true>), g, b, 0, st, pl, a);
    } else {
      if (grad) hipLaunchKernelGGL((k_hf_stream<true, false, true>), g, b, 0, st, pl, a);
      else hipLaunchKernelGGL((k_hf_stream<false, false, true>), g, b, 0, st, pl, a);
    }
  } else if (stat) {
    if (grad) hipLaunchKernelGGL((k_hf_stream<true, true, false>), g, b, 0, st, pl, a);
    else hipLaunchKernelGGL((k_hf_stream<false, true, false>), g, b, 0, st, pl, a);
  } else {
    if (grad) hipLaunchKernelGGL((k_hf_stream<true, false, false>), g, b, 0, st, pl, a);
    else hipLaunchKernelGGL((k_hf_stream<false, false, false>), g, b, 0, st, pl, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grad) hipLaunchKernelGGL((k_hf_finish<true>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
  else hipLaunchKernelGGL((k_hf_finish<false>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
  return hipGetLastError();
}

}  // namespace nllmi
