// kernels_dev.h -- the streaming NLL kernels for gfx950 (templates over the
// model shape).  Device code only: compiled ahead of time for the shapes of
// variants_*.hip, and at run time by hipRTC for any other shape.
//
//   k_single   one dataset: persistent grid, each block computes the
//              per-point constants itself, streams its tiles of the SoA
//              event columns once (coalesced, U events per thread per
//              tile), reduces in double-double and writes one record per
//              block.
//   k_single_finish  one block: the block records in block order, NLL
//              (and the gradient) to device memory; in a fit, the update.
//   k_single_fit  one gradient-descent step per launch: every block first
//              takes the previous step's update from that launch's records
//              (same bits in every block), then streams at the new proposal.
//   k_consts   per-set constants for many datasets (one block per set).
//   k_schedule tile counts per set and their prefix (one block).
//   k_sets     many datasets: work items (set, tile) over a persistent
//              grid, one double-double record per item.
//   k_sets_finish  one block per set, launched after k_sets: that set's
//              item records in item order, its NLL / gradient / status
//              and, when fitting, the gradient-descent step and the
//              constants of the next proposal (a batched fit step is these
//              two launches).
//   k_fit_init / k_fit_final   state set-up and read-out around the steps.
//
// No matrix cores: the pass is a streaming map-reduce.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "args.h"
#include "model.h"
#include "prologue.h"
#include "reduce.h"

namespace nllmi {

// ------------------------------------------------------------------------
// finisher: block totals -> NLL, status and gradient, by a whole block.
// pl, pt and theta are LDS copies.  Every thread forms NLL and status (the
// same bits everywhere); thread q < n_param forms d NLL / d theta_q from
//   sum_k T_k d log w_k/d theta_q
//     + sum_{l,p: param(l,p) = q} [ fscale_lp F_lp - Rtot_l d log Z_l/d theta_p ]
// with T_k = sum_i r_k, F_lp = sum_i R_l phi_lp and Rtot_l = sum_{k ∋ l} T_k
// (N for root leaves); the leaf and term loops are compile-time.
// Results: *s_nll, *s_st (thread 0 writes) and g[q], visible after the
// trailing barrier.  n: the number of events, or over weighted events the
// weights' sum W.
// ------------------------------------------------------------------------
template <class M, bool GRAD>
__device__ __forceinline__ void finish_block(const Plan& pl, const PerTheta& pt, const DD* tot, double n,
                                             const double* theta, bool flagged, double* s_nll, int* s_st, double* g) {
  constexpr int NA = M::template NA<GRAD>;
  const int64_t bad_events = (int64_t)(tot[NA].hi + tot[NA].lo);
  const double sum_l = tot[0].hi + tot[0].lo;
  // the FP32 pass sums log-densities without the term constants: croot +
  // ck_0 for every event, ck_k - ck_0 for every event whose largest term is k
  double cn = pt.croot;
  double cterms = 0.0;
  if constexpr (M::PREC == 1 && M::K > 1) {
    cn += pt.ck[0];
#pragma unroll
    for (int k = 1; k < M::K; ++k) {
      const DD c = tot[M::template CNT_BASE<GRAD> + k - 1];
      cterms += (pt.ck[k] - pt.ck[0]) * (c.hi + c.lo);
    }
  }
  double nll = -((sum_l + cterms) + n * cn);
  if (pl.extended) {
    const double nu = expected_count(pl, theta);
    nll += nu - n * log(nu);
  }
  int status = 0;
  if (flagged) status = -1;                                                 // malformed offsets
  else if (pt.bad & 1) status = -3;                                         // parameter range
  else if (pt.bad || bad_events > 0 || !__builtin_isfinite(nll)) status = -5;  // invalid density
  if (status != 0) nll = __builtin_inf();
  if (threadIdx.x == 0) {
    *s_nll = nll;
    *s_st = status;
  }
  if constexpr (GRAD) {
    const int q = threadIdx.x;
    if (q < pl.n_param) {
      double acc = 0.0;
      if (status == 0) {
        double T[M::K];
        double Tsum = 0.0;
#pragma unroll
        for (int k = 0; k < M::K - 1; ++k) {
          T[k] = tot[M::TERM_BASE + k].hi + tot[M::TERM_BASE + k].lo;
          Tsum += T[k];
        }
        T[M::K - 1] = M::K > 1 ? n - Tsum : 0.0;  // sum_k r_k = 1 per event
        if constexpr (M::K > 1) {
#pragma unroll
          for (int k = 0; k < M::K; ++k) acc += T[k] * pt.dlogw[k][q];
        }
        static_for<M::L>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          constexpr int off = M::template leaf_off<l>();
          double R = n;
          if constexpr (!M::ROOTs[l]) {
            const int mask_l = 1 << l;
            R = 0.0;
#pragma unroll
            for (int k = 0; k < M::K; ++k) R += (pl.term_mask[k] & mask_l) ? T[k] : 0.0;
          }
#pragma unroll
          for (int p = 0; p < M::NPs[l]; ++p) {
            if (pl.leaf_param[l][p] == q) {
              const DD v = tot[M::LEAF_BASE + off + p];
              double F = v.hi + v.lo;
              if constexpr (M::PREC == 1) F += pt.phioff[l][p] * R;  // features of x - x0
              acc += pt.fscale[l][p] * F - R * pt.dlogz[l][p];
            }
          }
        });
        acc = -acc;
        if (pl.extended && is_count_param(pl, q)) acc += 1.0 - n / expected_count(pl, theta);
      }
      g[q] = pl.par_free[q] ? acc : 0.0;
    }
  }
  __syncthreads();
}

// Gradient-descent state of set s as read at the start of a finishing
// kernel (f_acc, eta and the last status; thread q < P: its parameter's
// entries), so that these loads travel together with the kernel's other
// loads.  Every lane loads, with neither a branch nor a select after the
// load (threads q >= P read parameter 0's entries, which no caller uses),
// so that the waits that follow count these loads exactly.
struct GDPre {
  double fa, eta;         // every thread
  int ls;                 // every thread: last status
  double acc, ga, prop;   // thread q < P
};
__device__ inline GDPre gd_preload(const GDState& gd, int s, int P) {
  GDPre r;
  const int q = threadIdx.x;
  r.fa = gd.f_acc[s];
  r.eta = gd.eta[s];
  r.ls = gd.last_status[s];
  const size_t i = (size_t)s * P + (q < P ? q : 0);
  r.acc = gd.th_acc[i];
  r.ga = gd.g_acc[i];
  r.prop = gd.th_prop[i];
  return r;
}

// Gradient descent on the mean NLL with step halving, by a whole block:
// thread 0 accepts the evaluated proposal when its NLL is finite and exceeds
// the last accepted one by at most 4 ulps (rounding noise), else halves the
// step; then thread q forms the next proposal theta_acc - eta g_acc / N of
// parameter q (free parameters only), stores it and returns it (threads
// q >= P return 0).  st/nll are block-uniform LDS values; grad is in LDS.
__device__ inline double gd_update(const Plan& pl, const GDState& gd, int s, int st, double nll,
                                   const double* grad, double n_s, const GDPre& pre) {
  __shared__ int s_ok;
  __shared__ double s_step;
  const int P = pl.n_param;
  if (threadIdx.x == 0) {
    const double fa = pre.fa;
    const bool ok = st == 0 && __builtin_isfinite(nll) && nll <= fa + 4.0 * 2.220446049250313e-16 * fabs(fa);
    double eta = pre.eta;
    if (ok) {
      gd.f_acc[s] = nll;
      gd.last_status[s] = 0;
    } else {
      eta *= 0.5;
      gd.eta[s] = eta;
      if (!__builtin_isfinite(fa)) gd.last_status[s] = st != 0 ? st : -5;
    }
    s_ok = ok;
    s_step = eta / (n_s > 0.0 ? n_s : 1.0);
  }
  __syncthreads();
  const int q = threadIdx.x;
  double next = 0.0;
  if (q < P) {
    double acc = pre.acc, ga = pre.ga;
    if (s_ok) {
      acc = pre.prop;
      ga = grad[q];
      gd.th_acc[(size_t)s * P + q] = acc;
      gd.g_acc[(size_t)s * P + q] = ga;
    }
    next = pl.par_free[q] ? acc - s_step * ga : acc;
    gd.th_prop[(size_t)s * P + q] = next;
  }
  return next;
}

// The same step for a state kept in two buffers (by step parity): the
// state is read from pre (gd_preload of the input buffer) and, when
// `writer`, every field is written to `out`, changed or not.  Threads
// q >= P return 0.  Every block of a streaming launch calls it with the
// same inputs (same bits everywhere); only one writes.
__device__ inline double gd_update_to(const Plan& pl, const GDState& out, int st, double nll, const double* grad,
                                      double n_s, const GDPre& pre, bool writer) {
  __shared__ int s_ok;
  __shared__ double s_step;
  const int P = pl.n_param;
  if (threadIdx.x == 0) {
    const double fa = pre.fa;
    const bool ok = st == 0 && __builtin_isfinite(nll) && nll <= fa + 4.0 * 2.220446049250313e-16 * fabs(fa);
    double eta = pre.eta, f = fa;
    int ls = pre.ls;
    if (ok) {
      f = nll;
      ls = 0;
    } else {
      eta *= 0.5;
      if (!__builtin_isfinite(fa)) ls = st != 0 ? st : -5;
    }
    if (writer) {
      out.f_acc[0] = f;
      out.eta[0] = eta;
      out.last_status[0] = ls;
    }
    s_ok = ok;
    s_step = eta / (n_s > 0.0 ? n_s : 1.0);
  }
  __syncthreads();
  const int q = threadIdx.x;
  double next = 0.0;
  if (q < P) {
    const double acc = s_ok ? pre.prop : pre.acc;
    const double ga = s_ok ? grad[q] : pre.ga;
    next = pl.par_free[q] ? acc - s_step * ga : acc;
    if (writer) {
      out.th_acc[q] = acc;
      out.g_acc[q] = ga;
      out.th_prop[q] = next;
    }
  }
  return next;
}

// ------------------------------------------------------------------------
// BHHH: B = sum_i s_i s_i^T of the events' scores s_i = d log p(x_i)/d theta
// (Berndt, Hall, Hall and Hausman), the outer-product approximation of the
// NLL's Hessian, and the damped (Levenberg-Marquardt) step on it.
// ------------------------------------------------------------------------
// index of the second moment of score features (i, j), i <= j, in the
// upper-triangle row order of AccBhhh
template <int NVF>
__device__ __forceinline__ int mom_index(int i, int j) {
  return i * NVF - i * (i - 1) / 2 + (j - i);
}

// B (LDS, P x P row-major, symmetric) from the reduced totals: the score is
// affine in the features, s_i = c0 + A v_i, with, for parameter q,
//   A[q][k]         = d log w_k/d theta_q - sum_{non-root l in S_k, p -> q} d log Z_lp
//   A[q][NT+off+p]  = fscale_lp             (leaf l's local parameter p is q)
//   c0[q]           = - sum_{root l, p -> q} d log Z_lp,
// so B = N c0 c0^T + c0 (A m1)^T + (A m1) c0^T + A M2 A^T with m1 = sum v and
// M2 = sum v v^T; plus N / nu^2 at every pair of the parameters that make
// the expected count nu of an extended model.  Rows and
// columns of fixed parameters, and everything after an invalid evaluation,
// are 0.  Every entry is formed for (min, max) of its indices, so B is
// exactly symmetric.  Ends with a barrier.
template <class M>
__device__ __forceinline__ void bhhh_assemble(const Plan& pl, const PerTheta& pt, const DD* tot, int64_t n,
                                              const double* theta, int st, double* B) {
  using AB = AccBhhh<M>;
  constexpr int NT = AB::NT, NVF = AB::NVF, NA = AB::NA;
  __shared__ double sA[kMaxParams][NVF];
  __shared__ double sc0[kMaxParams], sAm1[kMaxParams];
  const int P = pl.n_param, t = threadIdx.x;
  const double dn = (double)n;
  if (t < P) {
    const int q = t;
    double Aq[NVF];
#pragma unroll
    for (int j = 0; j < NVF; ++j) Aq[j] = 0.0;
    double c0 = 0.0;
    if constexpr (NT > 0) {
#pragma unroll
      for (int k = 0; k < M::K; ++k) Aq[k] = pt.dlogw[k][q];
    }
    static_for<M::L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      constexpr int off = M::template leaf_off<l>();
#pragma unroll
      for (int p = 0; p < M::NPs[l]; ++p) {
        if (pl.leaf_param[l][p] == q) {
          Aq[NT + off + p] += pt.fscale[l][p];
          if constexpr (M::ROOTs[l]) {
            c0 -= pt.dlogz[l][p];
          } else {
#pragma unroll
            for (int k = 0; k < M::K; ++k)
              if ((pl.term_mask[k] >> l) & 1) Aq[k] -= pt.dlogz[l][p];
          }
        }
      }
    });
    double m1[NVF];
    if constexpr (NT > 0) {
      double Tsum = 0.0;
#pragma unroll
      for (int k = 0; k < M::K - 1; ++k) {
        m1[k] = tot[M::TERM_BASE + k].hi + tot[M::TERM_BASE + k].lo;
        Tsum += m1[k];
      }
      m1[M::K - 1] = dn - Tsum;
    }
#pragma unroll
    for (int j = 0; j < M::NPT; ++j) m1[NT + j] = tot[M::LEAF_BASE + j].hi + tot[M::LEAF_BASE + j].lo;
    double am = 0.0;
#pragma unroll
    for (int j = 0; j < NVF; ++j) {
      am = fma(Aq[j], m1[j], am);
      sA[q][j] = Aq[j];
    }
    sc0[q] = c0;
    sAm1[q] = am;
  }
  __syncthreads();
  for (int e = t; e < P * P; e += blockDim.x) {
    const int q0 = e / P, r0 = e - q0 * P;
    const int q = q0 < r0 ? q0 : r0, r = q0 < r0 ? r0 : q0;
    double b = 0.0;
    if (st == 0 && pl.par_free[q] && pl.par_free[r]) {
      double quad = 0.0;
#pragma unroll
      for (int i = 0; i < NVF; ++i) {
        double row = 0.0;  // (M2 A_r^T)_i
#pragma unroll
        for (int j = 0; j < NVF; ++j) {
          const DD mm = tot[NA + 1 + (i <= j ? mom_index<NVF>(i, j) : mom_index<NVF>(j, i))];
          row = fma(mm.hi + mm.lo, sA[r][j], row);
        }
        quad = fma(sA[q][i], row, quad);
      }
      b = ((dn * sc0[q]) * sc0[r] + sc0[q] * sAm1[r]) + (sAm1[q] * sc0[r] + quad);
      if (pl.extended && is_count_param(pl, q) && is_count_param(pl, r)) {
        const double nu = expected_count(pl, theta);
        b += dn / (nu * nu);
      }
    }
    B[e] = b;
  }
  __syncthreads();
}

// Solve (B + lambda D) d = -g over the free parameters by Cholesky, D the
// diagonal of B floored at 1e-12 of its largest free entry; fixed
// parameters enter as identity rows (d = 0), which leaves the free part's
// arithmetic unchanged.  One thread; L is P x P scratch (LDS).  False if the
// damped matrix is not positive definite.
__device__ inline bool damped_solve(const Plan& pl, const double* B, const double* g, double lambda, double* d,
                                    double* L) {
  const int P = pl.n_param;
  double dmax = 0.0;
  for (int k = 0; k < P; ++k)
    if (pl.par_free[k]) dmax = fmax(dmax, B[k * P + k]);
  for (int a = 0; a < P; ++a) {
    for (int b = 0; b <= a; ++b) {
      double s;
      if (!pl.par_free[a] || !pl.par_free[b]) {
        s = a == b ? 1.0 : 0.0;
      } else {
        s = B[a * P + b];
        if (a == b) s += lambda * fmax(s, 1e-12 * dmax);
      }
      for (int c = 0; c < b; ++c) s -= L[a * P + c] * L[b * P + c];
      if (a == b) {
        if (!(s > 0.0) || !__builtin_isfinite(s)) return false;
        L[a * P + a] = sqrt(s);
      } else {
        L[a * P + b] = s / L[b * P + b];
      }
    }
  }
  for (int a = 0; a < P; ++a) {  // L y = -g  (y kept in d)
    double s = pl.par_free[a] ? -g[a] : 0.0;
    for (int c = 0; c < a; ++c) s -= L[a * P + c] * d[c];
    d[a] = s / L[a * P + a];
  }
  for (int a = P - 1; a >= 0; --a) {  // L^T d = y
    double s = d[a];
    for (int c = a + 1; c < P; ++c) s -= L[c * P + a] * d[c];
    d[a] = s / L[a * P + a];
  }
  return true;
}

// Damped BHHH step by a whole block (set 0): thread 0 accepts the
// evaluated proposal when its NLL is finite and at most 4 ulps above the
// last accepted one (lambda /= 10, floored at 1e-12), else lambda *= 10;
// the accepted point, gradient and matrix are kept (B, LDS, becomes the
// accepted matrix; bpre is this thread's entry of the previously accepted
// one); thread 0 solves the damped system, retrying with ten times the
// damping at most 8 times; thread q < P stores and returns its parameter of
// the next proposal (theta_acc if no solve succeeded), threads q >= P 0.
__device__ inline double bhhh_update(const Plan& pl, const GDState& gd, int st, double nll, const double* grad,
                                     double* B, double bpre, const GDPre& pre) {
  __shared__ int s_ok, s_solved;
  __shared__ double s_lam;
  __shared__ double s_acc[kMaxParams], s_g[kMaxParams], s_d[kMaxParams];
  __shared__ double s_L[kMaxParams * kMaxParams];
  const int P = pl.n_param, t = threadIdx.x;
  if (t == 0) {
    const double fa = pre.fa;
    const bool ok = st == 0 && __builtin_isfinite(nll) && nll <= fa + 4.0 * 2.220446049250313e-16 * fabs(fa);
    double lam = pre.eta;
    if (ok) {
      gd.f_acc[0] = nll;
      gd.last_status[0] = 0;
      lam = fmax(lam * 0.1, 1e-12);
    } else {
      lam *= 10.0;
      if (!__builtin_isfinite(fa)) gd.last_status[0] = st != 0 ? st : -5;
    }
    s_ok = ok;
    s_lam = lam;
  }
  __syncthreads();
  const bool ok = s_ok;
  if (t < P) {
    double acc = pre.acc, ga = pre.ga;
    if (ok) {
      acc = pre.prop;
      ga = grad[t];
      gd.th_acc[t] = acc;
      gd.g_acc[t] = ga;
    }
    s_acc[t] = acc;
    s_g[t] = ga;
  }
  if (t < P * P) {
    if (ok) gd.b_acc[t] = B[t];
    else B[t] = bpre;
  }
  __syncthreads();
  if (t == 0) {
    double lam = s_lam;
    bool solved = false;
    for (int tries = 0; tries < 8 && !solved; ++tries) {
      solved = damped_solve(pl, B, s_g, lam, s_d, s_L);
      if (!solved) lam *= 10.0;
    }
    gd.eta[0] = lam;
    s_solved = solved;
  }
  __syncthreads();
  double next = 0.0;
  if (t < P) {
    next = s_solved && pl.par_free[t] ? s_acc[t] + s_d[t] : s_acc[t];
    gd.th_prop[t] = next;
  }
  return next;
}

// ------------------------------------------------------------------------
// per-tile event loops
// ------------------------------------------------------------------------
// Event loads.  NT: non-temporal (the nt bit), for passes over more data
// than the last-level cache holds: a plain read over 4 GiB reaches
// ~7.3 TB/s on MI355X with it against ~6.4 TB/s with the default policy;
// data that stay cache-resident between passes (a single dataset of tens
// of MB evaluated again and again by a minimiser) are read faster with the
// default policy (the 1e7-event mixture's pass: ~5 % slower with NT).
template <bool NT>
__device__ __forceinline__ double ld_event(const double* p) {
  if constexpr (NT) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

template <class M, int U, bool NT = false>
__device__ inline void load_tile(const double* const* cols, int64_t base, double (&x)[U][M::NOBS]) {
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int o = 0; o < M::NOBS; ++o) x[u][o] = ld_event<NT>(&cols[o][base + (int64_t)u * kBlock]);
}

template <class M, bool GRAD, int U, class CT, class AT>
__device__ inline void compute_tile(const double (&x)[U][M::NOBS], const CT& C, AT& acc) {
  acc.begin_tile();
#pragma unroll
  for (int u = 0; u < U; ++u) model_event<M, GRAD>(x[u], C, acc);
  acc.end_tile();
}

// Full tiles base0, base0 + stride, ... (count of them), software
// pipelined through a ring of R register buffers: the first R - 1 tiles
// arrive preloaded in xb[0 .. R-2], and before tile k is computed the loads
// of tile k + R - 1 are issued into the buffer that tile k - 1 used, so each
// load has R - 1 tiles of compute to arrive.  The ring is unrolled (buffers
// rotate without copies).  The main loop runs over groups of R tiles whose
// loads all stay in range, with no branches, so that the compiler's
// load-counter waits see every load of the ring in flight; the last tiles
// (fewer than 2R) test their loads one by one.  Three buffers for shapes
// with at most 8 accumulators; two for the heavier ones, whose registers
// are already scarce (measured: three cost the 2-D model ~4-5 %, two cost
// the mixture at 1e8 events ~18 %).
template <class M>
constexpr int ring_depth() {
  return M::template NA<true> <= 8 ? 3 : 2;
}

template <class M, int U, int R, bool NT = false>
__device__ inline void preload_ring(const double* const* cols, int64_t base0, int64_t stride, int64_t count,
                                    double (&xb)[R][U][M::NOBS]) {
#pragma unroll
  for (int j = 0; j < R - 1; ++j)
    if (j < count) load_tile<M, U, NT>(cols, base0 + j * stride, xb[j]);
}

// The same with every load issued: tiles past count read the word at dummy
// (any valid address; the values are never used), so that the waits of a
// kernel start that loads its inputs before these tiles and uses them
// after count exactly the loads in flight.
template <class M, int U, int R>
__device__ inline void preload_ring_all(const double* const* cols, int64_t base0, int64_t stride, int64_t count,
                                        const double* dummy, double (&xb)[R][U][M::NOBS]) {
#pragma unroll
  for (int j = 0; j < R - 1; ++j) {
    const bool in = j < count;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int o = 0; o < M::NOBS; ++o)
        xb[j][u][o] = *(in ? cols[o] + base0 + j * stride + (int64_t)u * kBlock : dummy);
  }
}

template <class M, bool GRAD, int U, int R, bool NT = false, class CT, class AT>
__device__ inline void stream_tiles(const double* const* cols, int64_t base0, int64_t stride, int64_t count,
                                    double (&xb)[R][U][M::NOBS], const CT& C, AT& acc) {
  // tile k sits in xb[k % R]; groups g < safe load tiles up to
  // safe * R + R - 2 <= count - 1
  const int64_t safe = count >= R - 1 ? (count - (R - 1)) / R : 0;
  for (int64_t g = 0; g < safe; ++g) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int64_t k = g * R + j;
      load_tile<M, U, NT>(cols, base0 + (k + R - 1) * stride, xb[(j + R - 1) % R]);
      compute_tile<M, GRAD, U>(xb[j], C, acc);
    }
  }
  // the remaining count - safe * R <= 2R - 2 tiles
#pragma unroll
  for (int j = 0; j < 2 * R - 2; ++j) {
    const int64_t k = safe * R + j;
    if (k < count) {
      if (k + R - 1 < count) load_tile<M, U, NT>(cols, base0 + (k + R - 1) * stride, xb[(j + R - 1) % R]);
      compute_tile<M, GRAD, U>(xb[j % R], C, acc);
    }
  }
}

template <class M, bool GRAD, int U, bool NT = false, class CT, class AT>
__device__ inline void stream_part_tile(const double* const* cols, int64_t base, int64_t end, const CT& C,
                                        AT& acc) {
  acc.begin_tile();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * kBlock;
    if (i < end) {
      double x[M::NOBS];
#pragma unroll
      for (int o = 0; o < M::NOBS; ++o) x[o] = ld_event<NT>(&cols[o][i]);
      model_event<M, GRAD>(x, C, acc);
    }
  }
  acc.end_tile();
}

// A leaf's per-point tables (kAuxWords words) copied by NT threads, no
// barrier.
template <int NT>
__device__ inline void copy_aux(double* dst, const double* __restrict__ src) {
  for (int i = threadIdx.x; i < kAuxWords; i += NT) dst[i] = src[i];
}

// ------------------------------------------------------------------------
// single dataset
// ------------------------------------------------------------------------
// Streaming pass over one dataset: per-block prologue, the block's tiles,
// one compensated partial per block (plain stores; the next kernel on the
// stream reads them).  Block 0 also leaves its per-point constants for the
// finishing kernel.
template <class M, bool GRAD, int U, bool FIT = false, bool BH = false>
__global__ __launch_bounds__(kBlock) void k_single(const Plan pl, const SingleArgs a) {
  static_assert(!BH || (GRAD && M::PREC == 0), "BHHH moments: FP64 gradient pass only");
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NM = BH ? AccBhhh<M>::NM : 0;  // BHHH second moments
  constexpr int NV = NA + 1 + NM;              // + invalid-event count
  constexpr int NR = NA + 1 > NM ? NA + 1 : NM;  // values per block_sum_vals pass
  __shared__ Plan spl;
  __shared__ double s_theta[kMaxParams];
  __shared__ PerTheta pt;
  __shared__ double red[NR * (kBlock + 1)];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_aux[M::AUX ? kAuxWords : 1];  // a leaf's per-point tables

  // Evaluation: plan and parameters first, then the first event tile
  // (which does not depend on theta), whose loads overlap the prologue.
  // Fit: the constants of the proposal were prepared by the previous step's
  // finishing kernel; the event pass reads the few it needs straight from
  // there (uniform loads), overlapping the first tiles' loads.
  // Every load is issued before the first LDS copy is written: plan
  // words and parameters, then the first event tiles.
  PlanRegs<kBlock> plr;
  double thv = 0.0;
  if constexpr (!FIT) {
    plr.load(pl);
    const int P = pl.n_param;
    const double v = a.theta[(int)threadIdx.x < P ? threadIdx.x : 0];
    thv = (int)threadIdx.x < P ? v : 0.0;
  }
  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];
  const int64_t tile = (int64_t)kBlock * U;
  const int64_t nfull = a.n / tile;
  const int64_t mine = nfull > (int64_t)blockIdx.x ? (nfull - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t base0 = (int64_t)blockIdx.x * tile + threadIdx.x;
  double xb[ring_depth<M>()][U][M::NOBS];
  preload_ring_all<M, U>(cols, base0, (int64_t)gridDim.x * tile, mine, a.glx, xb);
  if constexpr (!FIT) {
    plr.store(&spl);
    if ((int)threadIdx.x < pl.n_param) s_theta[threadIdx.x] = thv;
  }

  using CT = typename Pass<M, GRAD>::C;
  __shared__ double s_etab[CT::kExpTab ? kExpTabSize : 1];
  if constexpr (CT::kExpTab) stage_exp_table(s_etab);
  if constexpr (M::EVENT_LOG) stage_log_table(g_log_tab);
  CT C;
  int bad;
  if constexpr (FIT) {
    if constexpr (M::AUX) {
      copy_aux<kBlock>(s_aux, a.aux);
      __syncthreads();
    }
    C.load(*a.consts, pl, s_aux);
    bad = uniform(a.consts->bad);
  } else {
    compute_pertheta<M>(spl, s_theta, a.glx, a.glw, &pt, small, s_aux);
    C.load(pt, pl, s_aux);
    bad = uniform(pt.bad);
  }
  if constexpr (CT::kExpTab) C.etab = s_etab;
  if constexpr (CT::kExpTab || M::EVENT_LOG) __syncthreads();
  std::conditional_t<BH, AccBhhh<M>, typename Pass<M, GRAD>::A> acc;
  acc.init();
  if (bad == 0) {
    stream_tiles<M, GRAD, U>(cols, base0, (int64_t)gridDim.x * tile, mine, xb, C, acc);
    const int64_t rest = nfull * tile;
    if (rest < a.n && blockIdx.x == (unsigned)(nfull % gridDim.x))
      stream_part_tile<M, GRAD, U>(cols, rest + threadIdx.x, a.n, C, acc);
  }

  // partial record: the NA sums, the invalid-event count, the NM moments
  if constexpr (BH) {
    double w[NA + NM];
    acc.finalize(w);
    double v0[NA + 1], v1[NM];
#pragma unroll
    for (int j = 0; j < NA; ++j) v0[j] = w[j];
    v0[NA] = (double)acc.run.bad;
#pragma unroll
    for (int j = 0; j < NM; ++j) v1[j] = w[NA + j];
    block_sum_vals<NA + 1, kBlock>(v0, red, tot);
    block_sum_vals<NM, kBlock>(v1, red, tot + NA + 1);
  } else {
    double v[NV];
    acc.finalize(reinterpret_cast<double(&)[NA]>(v));
    v[NA] = (double)acc.bad;
    block_sum_vals<NV, kBlock>(v, red, tot);
  }
  if (threadIdx.x < NV) reinterpret_cast<DD*>(a.partials)[(size_t)blockIdx.x * NV + threadIdx.x] = tot[threadIdx.x];
  if (!FIT && blockIdx.x == 0) copy_pertheta<M, kBlock>(a.pt_out, &pt, pl.n_param);
}

// Finishing kernel (one block of kFinishBlock threads): the block partials
// in block order, then NLL and gradient; in fit mode the gradient-descent
// step of the proposal just evaluated and the per-point constants of the
// next proposal (for the next step's streaming kernel).  Every load it
// needs is issued at once at the start.
template <class M, bool GRAD, bool FIT = false, bool BH = false>
__global__ __launch_bounds__(kFinishBlock) void k_single_finish(const Plan pl, const SingleArgs a, int n_blocks) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1 + (BH ? AccBhhh<M>::NM : 0);
  __shared__ Plan spl;
  __shared__ DD tot[NV];
  __shared__ double s_grad[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_nll;
  __shared__ int s_st;
  __shared__ double small[(kFinishBlock / 64) * (kMaxLeafParams + 1)];
  const int t = threadIdx.x;
  stage_plan<kFinishBlock>(pl, &spl);
  PtRegs<M, kFinishBlock> ptv;
  ptv.load(FIT ? a.consts : a.pt_out, pl.n_param);
  stage_theta(FIT ? a.gd.th_prop : a.theta, pl.n_param, s_theta);
  GDPre pre{};
  if constexpr (FIT) pre = gd_preload(a.gd, 0, pl.n_param);
  double bpre = 0.0;  // BHHH fit: this thread's entry of the accepted matrix
  if constexpr (FIT && BH) {
    const int P = pl.n_param;
    if (t < P * P) bpre = a.gd.b_acc[t];
  }
  // the events' count, or the weights' sum W (attached with the weights)
  double neff = (double)a.n;
  if constexpr (M::WEIGHTED) neff = *a.wsum;
  // the gradient-descent steps (k_single_fit) store their records value-major
  std::conditional_t<FIT && !BH, RecordSumT<NV, kFinishBlock>, RecordSum<NV, kFinishBlock>> rs;
  rs.issue(reinterpret_cast<const DD*>(a.partials), n_blocks);
  ptv.store(&spt, pl.n_param);
  rs.reduce(reinterpret_cast<const DD*>(a.partials), n_blocks, tot);  // ends with a barrier
  finish_block<M, GRAD>(spl, spt, tot, neff, s_theta, false, &s_nll, &s_st, s_grad);
  __shared__ double s_B[BH ? kMaxParams * kMaxParams : 1];
  if constexpr (BH) bhhh_assemble<M>(spl, spt, tot, a.n, s_theta, s_st, s_B);
  if constexpr (FIT && !BH) {
    // after the last step of a gradient-descent fit (k_single_fit): that
    // step's update, into the other state buffer
    (void)gd_update_to(spl, a.gd_out, s_st, s_nll, s_grad, neff, pre, true);
  } else if constexpr (FIT) {
    const double next = bhhh_update(spl, a.gd, s_st, s_nll, s_grad, s_B, bpre, pre);
    if (t < spl.n_param) s_theta[t] = next;  // compute_pertheta starts with a barrier
    // the next proposal's constants, built in LDS (its phases read back
    // what other threads wrote) and stored with one parallel copy
    __shared__ double s_aux[M::AUX ? kAuxWords : 1];
    compute_pertheta<M, kFinishBlock>(spl, s_theta, a.glx, a.glw, &spt, small, s_aux);
    copy_pertheta<M, kFinishBlock>(a.consts, &spt, spl.n_param);
    if constexpr (M::AUX) copy_aux<kFinishBlock>(a.aux, s_aux);
  } else {
    if (t == 0) {
      *a.nll_out = s_nll;
      if (s_st == -3) atomicOr(a.status, (int)kStatusParam);
      if (s_st == -5) atomicOr(a.status, (int)kStatusPdf);
    }
    if (GRAD && a.grad_out && t < spl.n_param) a.grad_out[t] = s_grad[t];
    if constexpr (BH) {
      const int P = spl.n_param;
      if (a.bhhh_out && t < P * P) a.bhhh_out[t] = s_B[t];
    }
  }
}

// One gradient-descent step over one dataset in one launch.  Every block
// first finishes the previous step itself: the previous launch's block
// records (stored value-major, summed in a fixed order), that
// proposal's NLL and gradient, the accept-or-halve update and the
// constants of the next proposal -- the same inputs and arithmetic in every
// block, so the same bits everywhere; block 0 stores the new state and
// constants.  Then the block streams its tiles at the new proposal.  State,
// constants and records alternate between two buffers by step parity, so
// that no block overwrites what another block of the same launch still
// reads; the launch boundary makes them visible to the next step.  The
// first step (partials_prev null) takes the constants k_fit_init made.
// This removes one kernel per step: the loads of the first event tiles are
// issued before the finishing work and arrive during it.
template <class M, int U>
__global__ __launch_bounds__(kBlock) void k_single_fit(const Plan pl, const SingleArgs a) {
  constexpr int NA = M::template NA<true>;
  constexpr int NV = NA + 1;  // + invalid-event count
  using CT = typename Pass<M, true>::C;
  __shared__ Plan spl;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_grad[kMaxParams];
  __shared__ PerTheta pt;
  __shared__ double red[NV * (kBlock + 1)];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_nll;
  __shared__ int s_st;
  __shared__ double s_etab[CT::kExpTab ? kExpTabSize : 1];
  __shared__ double s_aux[M::AUX ? kAuxWords : 1];  // a leaf's per-point tables
  const int t = threadIdx.x;
  const bool first = a.partials_prev == nullptr;

  // Every load is issued, in the order the values are needed (loads
  // complete in order), before the first LDS copy is written: plan, state
  // and the previous proposal's constants and records, then the first event
  // tiles; each copy then waits for its own loads only.  The first step (no
  // records yet) issues the same loads from buffers that exist and ignores
  // them, so that no branch stands between the loads.
  PlanRegs<kBlock> plr;
  plr.load(pl);
  const GDPre pre = gd_preload(a.gd, 0, pl.n_param);  // .prop: the proposal evaluated last
  double neff = (double)a.n;
  if constexpr (M::WEIGHTED) neff = *a.wsum;
  PtRegs<M, kBlock> ptv;
  ptv.load(a.consts, pl.n_param);
  const DD* rec = reinterpret_cast<const DD*>(first ? a.partials : a.partials_prev);
  RecordSumT<NV, kBlock, 16> rs;
  rs.issue(rec, gridDim.x);
  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];
  const int64_t tile = (int64_t)kBlock * U;
  const int64_t nfull = a.n / tile;
  const int64_t mine = nfull > (int64_t)blockIdx.x ? (nfull - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t base0 = (int64_t)blockIdx.x * tile + t;
  double xb[ring_depth<M>()][U][M::NOBS];
  preload_ring_all<M, U>(cols, base0, (int64_t)gridDim.x * tile, mine, a.glx, xb);
  plr.store(&spl);
  if (t < pl.n_param) s_theta[t] = pre.prop;
  if constexpr (CT::kExpTab) stage_exp_table(s_etab);
  if constexpr (M::EVENT_LOG) stage_log_table(g_log_tab);

  CT C;
  int bad;
  if (first) {
    if constexpr (M::AUX) {
      copy_aux<kBlock>(s_aux, a.aux);
      __syncthreads();
    }
    C.load(*a.consts, pl, s_aux);
    bad = uniform(a.consts->bad);
  } else {
    ptv.store(&pt, pl.n_param);
    rs.reduce(rec, gridDim.x, tot);  // ends with a barrier
    finish_block<M, true>(spl, pt, tot, neff, s_theta, false, &s_nll, &s_st, s_grad);
    const double next = gd_update_to(spl, a.gd_out, s_st, s_nll, s_grad, neff, pre, blockIdx.x == 0);
    if (t < spl.n_param) s_theta[t] = next;  // compute_pertheta starts with a barrier
    compute_pertheta<M>(spl, s_theta, a.glx, a.glw, &pt, small, s_aux);
    if (blockIdx.x == 0) copy_pertheta<M, kBlock>(a.consts_out, &pt, spl.n_param);
    C.load(pt, pl, s_aux);
    bad = uniform(pt.bad);
  }
  if constexpr (CT::kExpTab) C.etab = s_etab;
  __syncthreads();

  typename Pass<M, true>::A acc;
  acc.init();
  if (bad == 0) {
    stream_tiles<M, true, U>(cols, base0, (int64_t)gridDim.x * tile, mine, xb, C, acc);
    const int64_t rest = nfull * tile;
    if (rest < a.n && blockIdx.x == (unsigned)(nfull % gridDim.x))
      stream_part_tile<M, true, U>(cols, rest + t, a.n, C, acc);
  }
  double v[NV];
  acc.finalize(reinterpret_cast<double(&)[NA]>(v));
  v[NA] = (double)acc.bad;
  block_sum_vals<NV, kBlock>(v, red, tot);
  if (t < NV) reinterpret_cast<DD*>(a.partials)[(size_t)t * gridDim.x + blockIdx.x] = tot[t];  // value-major
}

// ------------------------------------------------------------------------
// many datasets
// ------------------------------------------------------------------------
template <class M>
__global__ __launch_bounds__(kBlock) void k_consts(const Plan pl, const double* __restrict__ theta,
                                                  int n_sets, PerTheta* __restrict__ out,
                                                  double* __restrict__ aux_out,
                                                  const double* __restrict__ glx,
                                                  const double* __restrict__ glw) {
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ Plan spl;
  __shared__ double s_theta[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_aux[M::AUX ? kAuxWords : 1];
  const int s = blockIdx.x;
  if (s >= n_sets) return;
  stage_plan<kBlock>(pl, &spl);
  stage_theta(theta + (size_t)s * pl.n_param, pl.n_param, s_theta);
  compute_pertheta<M>(spl, s_theta, glx, glw, &spt, small, s_aux);
  copy_pertheta<M, kBlock>(&out[s], &spt, spl.n_param);
  if constexpr (M::AUX) copy_aux<kBlock>(aux_out + (size_t)s * kAuxWords, s_aux);
}

// items, consts and chunk_first also come as kernel arguments of their
// own: read-only and not aliased by anything the kernel writes, their
// uniform loads (item descriptors, a set's constants, the chunk table) go
// through the scalar unit and do not make the vector-load counter waits
// drain the ring.
template <class M, bool GRAD, int U>
__global__ __launch_bounds__(kBlock) void k_sets(const Plan pl, const SetsArgs a,
                                                 const WorkItem* __restrict__ items,
                                                 const PerTheta* __restrict__ consts,
                                                 const int64_t* __restrict__ chunk_first) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;
  __shared__ double red[NV * (kBlock + 1)];
  __shared__ DD tot[NV];
  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];
  using CT = typename Pass<M, GRAD>::C;
  __shared__ double s_etab[CT::kExpTab ? kExpTabSize : 1];
  __shared__ double s_aux[M::AUX ? kAuxWords : 1];  // a leaf's per-point tables (per item)
  if constexpr (CT::kExpTab) stage_exp_table(s_etab);
  if constexpr (M::EVENT_LOG) stage_log_table(g_log_tab);
  if constexpr (CT::kExpTab || M::EVENT_LOG) __syncthreads();

  // Block b streams the items of its chunks b, G + b, ..., (K-1) G + b in
  // turn (every block the same number of events; at any time the grid
  // reads neighbouring chunks).  Its items form one sequence of tiles (an
  // item of len events has max(1, ceil(len / (256 U))) tiles, its last one
  // partial), streamed through one ring of R register buffers that runs
  // across item boundaries: a load cursor issues the loads of tile k + R - 1
  // while a compute cursor evaluates tile k, so loads stay in flight
  // through an item's last tiles, its block reduction and the switch to the
  // next item's constants.  Every tile issues its U x NOBS loads
  // unconditionally (lanes past an item's end, empty items and the ring's
  // run-out read a dummy word of the Gauss-Legendre table), so that the
  // compiler's load-counter waits see the whole ring in flight; events past
  // an item's end are masked in the arithmetic.  Non-temporal loads: the
  // sets together are read once per pass (a batch of toys is GBs).
  constexpr int R = ring_depth<M>();
  const int64_t step = (int64_t)kBlock * U;
  const double* dummy = a.glx;
  auto ntiles = [&](const WorkItem& w) -> int64_t {
    const int64_t len = w.end - w.start;
    return len > 0 ? (len + step - 1) / step : 1;
  };
  // a position in the block's item sequence: item i of the chunk of round
  // r (items chunk_first[j] .. chunk_first[j+1] - 1, j = r G + b)
  struct Seq {
    int64_t i, ie;
    int r;
  };
  const int64_t G = gridDim.x;
  const int K = a.rounds;
  auto settle = [&](Seq& q) -> bool {  // skip chunks without items; false at the end
    while (q.i >= q.ie) {
      if (++q.r >= K) return false;
      q.i = chunk_first[(int64_t)q.r * G + blockIdx.x];
      q.ie = chunk_first[(int64_t)q.r * G + blockIdx.x + 1];
    }
    return true;
  };
  Seq q0{chunk_first[blockIdx.x], chunk_first[blockIdx.x + 1], 0};
  const bool any = settle(q0);
  double xb[R][U][M::NOBS];

  // load cursor (R - 1 tiles ahead of the compute cursor)
  Seq lnq = q0;
  bool l_live = any, ln_live = false;
  int64_t l_tile = 0, l_T = 1;
  WorkItem l_w{0, 0, 0, 0}, l_next{0, 0, 0, 0};
  if (l_live) {
    l_w = items[q0.i];
    l_T = ntiles(l_w);
    ++lnq.i;
    ln_live = settle(lnq);
    if (ln_live) l_next = items[lnq.i];
  }
  auto issue = [&](double (&buf)[U][M::NOBS]) {
    const int64_t base = l_w.start + l_tile * step + threadIdx.x;
    const bool live = l_live;
    const bool full = live && l_w.end - (l_w.start + l_tile * step) >= step;
    const double* ptr[U][M::NOBS];
    if (full) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int o = 0; o < M::NOBS; ++o) ptr[u][o] = cols[o] + base + (int64_t)u * kBlock;
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + (int64_t)u * kBlock;
        const bool ok = live && i < l_w.end;
#pragma unroll
        for (int o = 0; o < M::NOBS; ++o) ptr[u][o] = ok ? cols[o] + i : dummy;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int o = 0; o < M::NOBS; ++o) buf[u][o] = ld_event<true>(ptr[u][o]);
    if (live && ++l_tile == l_T) {
      l_live = ln_live;
      l_w = l_next;
      l_T = ntiles(l_w);
      l_tile = 0;
      if (l_live) {
        ++lnq.i;
        ln_live = settle(lnq);
        if (ln_live) l_next = items[lnq.i];
      }
    }
  };

  // compute cursor
  Seq cq = q0, cnq = q0;
  bool c_live = any, cn_live = false;
  int64_t c_tile = 0, c_T = 1;
  WorkItem c_w{0, 0, 0, 0}, c_next{0, 0, 0, 0};
  CT C;
  bool skip = true;
  typename Pass<M, GRAD>::A acc;
  acc.init();
  auto enter = [&]() {  // constants of the item at cq (block-uniform)
    c_T = ntiles(c_w);
    c_tile = 0;
    cnq = cq;
    ++cnq.i;
    cn_live = settle(cnq);
    if (cn_live) c_next = items[cnq.i];
    const PerTheta& pt = consts[c_w.set];
    if constexpr (M::AUX) {  // the previous item's reads ended in its block sum
      copy_aux<kBlock>(s_aux, a.aux + (size_t)c_w.set * kAuxWords);
      __syncthreads();
    }
    C.load(pt, pl, s_aux);
    C.etab = s_etab;
    skip = uniform(pt.bad) != 0 || c_w.flag != 0;
    acc.init();
  };
  if (c_live) {
    c_w = items[cq.i];
    enter();
  }

#pragma unroll
  for (int j = 0; j < R - 1; ++j) issue(xb[j]);
  while (c_live) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      issue(xb[(j + R - 1) % R]);
      if (c_live) {
        if (!skip) {
          const int64_t t0 = c_w.start + c_tile * step;
          if (c_w.end - t0 >= step) {
            compute_tile<M, GRAD, U>(xb[j], C, acc);
          } else {
            acc.begin_tile();
#pragma unroll
            for (int u = 0; u < U; ++u)
              if (t0 + threadIdx.x + (int64_t)u * kBlock < c_w.end) model_event<M, GRAD>(xb[j][u], C, acc);
            acc.end_tile();
          }
        }
        if (++c_tile == c_T) {  // the item's record
          double v[NV];
          acc.finalize(reinterpret_cast<double(&)[NA]>(v));
          v[NA] = (double)acc.bad;
          block_sum_vals<NV, kBlock>(v, red, tot);
          if (threadIdx.x < NV)
            reinterpret_cast<DD*>(a.partials)[(size_t)cq.i * NV + threadIdx.x] = tot[threadIdx.x];
          cq = cnq;
          c_live = cn_live;
          if (c_live) {
            c_w = c_next;
            enter();
          }
        }
      }
    }
  }
}

// One block per set: reduce the set's work-item partials in item order,
// write NLL / gradient / status, or (fitting) take the gradient-descent step
// and prepare the constants of the next proposal.
// Threads per block of the per-set finishing kernel: 128 for models of at
// most 4 leaves without per-point tables (then the 4096 blocks of a large
// batch are all resident at once: two waves each), else 256.  The
// launchers use the same rule (kernels_impl.h, rtc.cpp).
template <class M>
constexpr int finish_threads() {
  return (M::AUX || M::L > 4) ? kBlock : kBlock / 2;
}
// Waves per SIMD the finishing kernel is compiled for: 8 (at most 64
// registers, so that 16 blocks of 128 threads share a CU) for one-leaf
// Gaussian, exponential and Chebyshev models, measured to fit that without
// spilling to scratch memory; else no requirement.
template <class M>
constexpr int finish_waves() {
  if constexpr (M::L == 1 && !M::AUX) {
    constexpr int k = M::template S<0>::Leaf::kKind;
    return (k == kGauss || k == kExp || k == kCheb) ? 8 : 1;
  } else {
    return 1;
  }
}

template <class M, bool GRAD, bool FIT>
__global__ __launch_bounds__(kBlock, finish_waves<M>()) void k_sets_finish(const Plan pl, const SetsArgs a) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;
  __shared__ Plan spl;
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_grad[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_nll;
  __shared__ int s_st;
  constexpr int NT = finish_threads<M>();  // the launch's threads per block
  const int s = blockIdx.x;  // the grid is exactly one block per set
  const int P = pl.n_param;
  const int t = threadIdx.x;
  // every independent load at once, before the first LDS copy is written:
  // plan, constants, parameters, fit state, the set's item range and
  // events, then its first batch of item records (each copy then waits for
  // its own loads only)
  PlanRegs<NT> plr;
  plr.load(pl);
  PtRegs<M, NT> ptv;
  ptv.load(&a.consts[s], P);
  GDPre pre{};
  double thv;
  if constexpr (FIT) {
    pre = gd_preload(a.gd, s, P);
    thv = pre.prop;
  } else {
    thv = a.theta[(size_t)s * P + (t < P ? t : 0)];  // read by every lane, kept by t < P
  }
  const int64_t first = a.tile_off[s], n_items = a.tile_off[s + 1] - first;
  const int flag = a.set_flag[s];
  const int64_t o0 = a.offsets[s], o1 = a.offsets[s + 1];
  const DD* recs = reinterpret_cast<const DD*>(a.partials) + (size_t)first * NV;
  RecordSum<NV, NT> rs;
  rs.issue(recs, n_items);
  plr.store(&spl);
  if (t < P) s_theta[t] = thv;
  ptv.store(&spt, P);
  rs.reduce(recs, n_items, tot);  // ends with a barrier
  const int64_t n_s = flag ? 0 : o1 - o0;
  finish_block<M, GRAD>(spl, spt, tot, n_s, s_theta, flag != 0, &s_nll, &s_st, s_grad);
  if constexpr (!FIT) {
    if (t == 0) {
      a.nll_out[s] = s_nll;
      if (a.status_out) a.status_out[s] = s_st;
    }
    if (GRAD && a.grad_out && t < P) a.grad_out[(size_t)s * P + t] = s_st == 0 ? s_grad[t] : 0.0;
  } else {
    const double next = gd_update(spl, a.gd, s, s_st, s_nll, s_grad, n_s, pre);
    if (t < P) s_theta[t] = next;  // compute_pertheta starts with a barrier
    __shared__ double s_aux[M::AUX ? kAuxWords : 1];
    compute_pertheta<M, NT>(spl, s_theta, a.glx, a.glw, &spt, small, s_aux);
    copy_pertheta<M, NT>(&a.consts[s], &spt, P);
    if constexpr (M::AUX) copy_aux<NT>(a.aux + (size_t)s * kAuxWords, s_aux);
  }
}

template <class M>
__global__ __launch_bounds__(kBlock) void k_fit_init(const Plan pl, const double* __restrict__ theta,
                                                    int n_sets, double eta, GDState gd,
                                                    PerTheta* __restrict__ consts,
                                                    double* __restrict__ aux,
                                                    const double* __restrict__ glx,
                                                    const double* __restrict__ glw) {
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ Plan spl;
  __shared__ double s_theta[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_aux[M::AUX ? kAuxWords : 1];
  const int s = blockIdx.x;
  if (s >= n_sets) return;
  const int P = pl.n_param;
  stage_plan<kBlock>(pl, &spl);
  if (threadIdx.x < P) {
    const double v = theta[(size_t)s * P + threadIdx.x];
    s_theta[threadIdx.x] = v;
    gd.th_acc[(size_t)s * P + threadIdx.x] = v;
    gd.th_prop[(size_t)s * P + threadIdx.x] = v;
    gd.g_acc[(size_t)s * P + threadIdx.x] = 0.0;
  }
  if (threadIdx.x == 0) {
    gd.f_acc[s] = __builtin_inf();
    gd.eta[s] = eta;
    gd.last_status[s] = 0;
  }
  if (gd.b_acc)
    for (int e = threadIdx.x; e < P * P; e += kBlock) gd.b_acc[(size_t)s * P * P + e] = 0.0;
  compute_pertheta<M>(spl, s_theta, glx, glw, &spt, small, s_aux);
  copy_pertheta<M, kBlock>(&consts[s], &spt, P);
  if constexpr (M::AUX) copy_aux<kBlock>(aux + (size_t)s * kAuxWords, s_aux);
}

// BHHH pass compiled: FP64 unweighted shapes with at most 6 score features
template <class M>
constexpr bool bh_compiled() {
  if constexpr (M::PREC != 0 || M::WEIGHTED) {
    return false;
  } else {
    return AccBhhh<M>::NVF <= 6;
  }
}

}  // namespace nllmi
