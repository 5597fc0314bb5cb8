// kernels_impl.h -- the streaming NLL kernels for gfx950 and their launchers
// (templates; instantiated per compiled model shape in variants_*.hip).
//
//   k_single   one dataset: persistent grid, each block computes the
//              per-point constants itself, streams its tiles of the SoA
//              event columns once (coalesced, U events per thread per
//              tile), reduces in double-double and the last block to finish
//              combines the block partials in block order and writes
//              NLL (and the gradient) to device memory.
//   k_consts   per-set constants for many datasets (one block per set).
//   k_schedule tile counts per set and their prefix (one block).
//   k_sets     many datasets: work items (set, tile) over a persistent
//              grid; the last item of a set to finish reduces that set's
//              partials in item order, writes its NLL / gradient / status
//              and, when fitting, performs the gradient-descent step and
//              prepares the constants of the next proposal.
//   k_fit_init / k_fit_final   state set-up and read-out around the steps.
//
// No matrix cores: the pass is a streaming map-reduce.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "model.h"
#include "prologue.h"
#include "reduce.h"

namespace nllmi {

// ------------------------------------------------------------------------
// finisher: totals -> NLL and gradient (thread 0 of one block).  The
// gradient is assembled in g (LDS, n_param entries) so that the scattered
// parameter indices never touch private memory.
// ------------------------------------------------------------------------
template <class M, bool GRAD>
__device__ int finish(const Plan& pl, const PerTheta& pt, const DD* tot, int64_t bad_events, int64_t n,
                      const double* theta, double* nll_out, double* g) {
  const int P = pl.n_param;
  const double sum_l = tot[0].hi + tot[0].lo;
  double nll = -(sum_l + (double)n * pt.croot);
  if (pl.extended) {
    const double nu = theta[pl.yield_param];
    nll += nu - (double)n * log(nu);
  }
  int status = 0;
  if (pt.bad) status = -3;                                                  // parameter range
  else if (bad_events > 0 || !__builtin_isfinite(nll)) status = -5;         // invalid density
  if (status != 0) nll = __builtin_inf();
  *nll_out = nll;
  if constexpr (GRAD) {
    #pragma unroll 1
    for (int q = 0; q < P; ++q) g[q] = 0.0;
    if (status != 0) return status;
    // per-event features: sum_i R_l phi_lp, times their scale; root leaves
    // carry -d log Z_l for every event
    #pragma unroll 1
    for (int l = 0, off = 0; l < pl.n_leaf; ++l) {
      #pragma unroll 1
      for (int p = 0; p < pl.leaf_np[l]; ++p, ++off) {
        const DD v = tot[M::LEAF_BASE + off];
        const int q = pl.leaf_param[l][p];
        g[q] += pt.fscale[l][p] * (v.hi + v.lo);
        if (pl.leaf_root[l]) g[q] -= (double)n * pt.dlogz[l][p];
      }
    }
    if constexpr (M::K > 1) {
      // sum_i r_k (d log w_k - sum_{non-root l in S_k} d log Z_l)
      #pragma unroll 1
      for (int k = 0; k < pl.n_term; ++k) {
        const double T = tot[M::TERM_BASE + k].hi + tot[M::TERM_BASE + k].lo;
        #pragma unroll 1
        for (int q = 0; q < P; ++q) g[q] += T * pt.dlogw[k][q];
        #pragma unroll 1
        for (int l = 0; l < pl.n_leaf; ++l)
          if (!pl.leaf_root[l] && ((pl.term_mask[k] >> l) & 1))
            #pragma unroll 1
            for (int p = 0; p < pl.leaf_np[l]; ++p) g[pl.leaf_param[l][p]] -= T * pt.dlogz[l][p];
      }
    }
    #pragma unroll 1
    for (int q = 0; q < P; ++q) g[q] = pl.par_free[q] ? -g[q] : 0.0;
    if (pl.extended && pl.par_free[pl.yield_param]) g[pl.yield_param] += 1.0 - (double)n / theta[pl.yield_param];
  }
  return status;
}

// ------------------------------------------------------------------------
// per-tile event loops
// ------------------------------------------------------------------------
template <class M, bool GRAD, int U>
__device__ inline void stream_full_tile(const double* const* cols, int64_t base, const Consts<M>& C,
                                        Acc<M, GRAD>& acc) {
  double x[U][M::NOBS];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int o = 0; o < M::NOBS; ++o) x[u][o] = cols[o][base + (int64_t)u * kBlock];
#pragma unroll
  for (int u = 0; u < U; ++u) model_event<M, GRAD>(x[u], C, acc);
  acc.renorm();
}

template <class M, bool GRAD, int U>
__device__ inline void stream_part_tile(const double* const* cols, int64_t base, int64_t end,
                                        const Consts<M>& C, Acc<M, GRAD>& acc) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * kBlock;
    if (i < end) {
      double x[M::NOBS];
#pragma unroll
      for (int o = 0; o < M::NOBS; ++o) x[o] = cols[o][i];
      model_event<M, GRAD>(x, C, acc);
    }
  }
  acc.renorm();
}

// ------------------------------------------------------------------------
// single dataset
// ------------------------------------------------------------------------
template <class M, bool GRAD, int U>
__global__ __launch_bounds__(kBlock) void k_single(const Plan pl, const SingleArgs a) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;  // + invalid-event count
  __shared__ PerTheta pt;
  __shared__ DD red[4 * NV];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_grad[kMaxParams];
  __shared__ int s_last;

  compute_pertheta<M>(pl, a.theta, a.glx, a.glw, &pt, small);
  Consts<M> C;
  C.load(pt, pl);
  Acc<M, GRAD> acc;
  acc.init();
  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];

  if (uniform(pt.bad) == 0) {
    const int64_t tile = (int64_t)kBlock * U;
    const int64_t nfull = a.n / tile;
    for (int64_t t = blockIdx.x; t < nfull; t += gridDim.x)
      stream_full_tile<M, GRAD, U>(cols, t * tile + threadIdx.x, C, acc);
    const int64_t rest = nfull * tile;
    if (rest < a.n && blockIdx.x == (unsigned)(nfull % gridDim.x))
      stream_part_tile<M, GRAD, U>(cols, rest + threadIdx.x, a.n, C, acc);
  }
  acc.close();

  DD v[NV];
#pragma unroll
  for (int j = 0; j < NA; ++j) v[j] = DD{acc.a[j], 0.0};
  v[NA] = DD{(double)acc.bad, 0.0};
  block_sum_dd<NV>(v, red, tot);
  if (threadIdx.x < NV) store_dd(&reinterpret_cast<DD*>(a.partials)[(size_t)blockIdx.x * NV + threadIdx.x], tot[threadIdx.x]);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(a.ticket, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  DD g[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) g[j] = DD{0.0, 0.0};
#pragma unroll 1
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
#pragma unroll
    for (int j = 0; j < NV; ++j) g[j] = dd_add(g[j], load_dd(&reinterpret_cast<const DD*>(a.partials)[(size_t)b * NV + j]));
  }
  block_sum_dd<NV>(g, red, tot);
  if (threadIdx.x == 0) {
    double nll;
    const int st = finish<M, GRAD>(pl, pt, tot, (int64_t)(tot[NA].hi + tot[NA].lo), a.n, a.theta, &nll, s_grad);
    *a.nll_out = nll;
    if (GRAD && a.grad_out)
      for (int q = 0; q < pl.n_param; ++q) a.grad_out[q] = s_grad[q];
    if (st == -3) atomicOr(a.status, (int)kStatusParam);
    if (st == -5) atomicOr(a.status, (int)kStatusPdf);
    __hip_atomic_store(a.ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------------
// many datasets
// ------------------------------------------------------------------------
template <class M>
__global__ __launch_bounds__(kBlock) void k_consts(const Plan pl, const double* __restrict__ theta,
                                                  int n_sets, PerTheta* __restrict__ out,
                                                  const double* __restrict__ glx,
                                                  const double* __restrict__ glw) {
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  const int s = blockIdx.x;
  if (s >= n_sets) return;
  compute_pertheta<M>(pl, theta + (size_t)s * pl.n_param, glx, glw, &out[s], small);
}

template <class M, bool GRAD, int U>
__global__ __launch_bounds__(kBlock) void k_sets(const Plan pl, const SetsArgs a) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;
  __shared__ DD red[4 * NV];
  __shared__ DD tot[NV];
  __shared__ int s_set;
  const int64_t total = a.tile_off[a.n_sets];
  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];

  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = a.n_sets;  // tile_off[lo] <= item < tile_off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.tile_off[mid] <= item) lo = mid;
        else hi = mid;
      }
      s_set = lo;
    }
    __syncthreads();
    const int s = uniform(s_set);
    const PerTheta& pt = a.consts[s];
    const int flag = a.set_flag[s];
    const int64_t start = (flag ? 0 : a.offsets[s]) + (item - a.tile_off[s]) * a.tile;
    const int64_t end = flag ? 0 : min(start + a.tile, a.offsets[s + 1]);

    Consts<M> C;
    C.load(pt, pl);
    Acc<M, GRAD> acc;
    acc.init();
    if (uniform(pt.bad) == 0 && flag == 0) {
      const int64_t step = (int64_t)kBlock * U;
      int64_t base = start;
      for (; base + step <= end; base += step) stream_full_tile<M, GRAD, U>(cols, base + threadIdx.x, C, acc);
      if (base < end) stream_part_tile<M, GRAD, U>(cols, base + threadIdx.x, end, C, acc);
    }
    acc.close();
    DD v[NV];
#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = DD{acc.a[j], 0.0};
    v[NA] = DD{(double)acc.bad, 0.0};
    block_sum_dd<NV>(v, red, tot);
    if (threadIdx.x < NV) reinterpret_cast<DD*>(a.partials)[(size_t)item * NV + threadIdx.x] = tot[threadIdx.x];
  }
}

// One block per set: reduce the set's work-item partials in item order,
// write NLL / gradient / status, or (fitting) take the gradient-descent step
// and prepare the constants of the next proposal.
template <class M, bool GRAD, bool FIT>
__global__ __launch_bounds__(kBlock) void k_sets_finish(const Plan pl, const SetsArgs a) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;
  __shared__ DD red[4 * NV];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_grad[kMaxParams];
  const int s = blockIdx.x;
  if (s >= a.n_sets) return;
  const int P = pl.n_param;
  const int64_t first = a.tile_off[s], n_items = a.tile_off[s + 1] - first;
  DD g[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) g[j] = DD{0.0, 0.0};
#pragma unroll 1
  for (int64_t it = threadIdx.x; it < n_items; it += kBlock) {
    const DD* src = reinterpret_cast<const DD*>(a.partials) + (size_t)(first + it) * NV;
#pragma unroll
    for (int j = 0; j < NV; ++j) g[j] = dd_add(g[j], src[j]);
  }
  block_sum_dd<NV>(g, red, tot);
  const int flag = a.set_flag[s];
  const int64_t n_s = flag ? 0 : a.offsets[s + 1] - a.offsets[s];
  const double* th = FIT ? a.gd.th_prop + (size_t)s * P : a.theta + (size_t)s * P;
  if (threadIdx.x == 0) {
    double nll;
    int st = finish<M, GRAD>(pl, a.consts[s], tot, (int64_t)(tot[NA].hi + tot[NA].lo), n_s, th, &nll, s_grad);
    if (flag) {
      st = -1;
      nll = __builtin_inf();
    }
    if constexpr (!FIT) {
      a.nll_out[s] = nll;
      if (GRAD && a.grad_out)
        for (int q = 0; q < P; ++q) a.grad_out[(size_t)s * P + q] = st == 0 ? s_grad[q] : 0.0;
      if (a.status_out) a.status_out[s] = st;
    } else {
      // gradient descent on the mean NLL, halving the step on a rejection
      double* th_acc = a.gd.th_acc + (size_t)s * P;
      double* g_acc = a.gd.g_acc + (size_t)s * P;
      double* th_prop = a.gd.th_prop + (size_t)s * P;
      // an increase of at most 4 ulps of the NLL is rounding noise, not an increase
      const double fa = a.gd.f_acc[s];
      const bool ok = st == 0 && __builtin_isfinite(nll) && nll <= fa + 4.0 * 2.220446049250313e-16 * fabs(fa);
      if (ok) {
        for (int q = 0; q < P; ++q) {
          th_acc[q] = th_prop[q];
          g_acc[q] = s_grad[q];
        }
        a.gd.f_acc[s] = nll;
        a.gd.last_status[s] = 0;
      } else {
        a.gd.eta[s] *= 0.5;
        if (!__builtin_isfinite(a.gd.f_acc[s])) a.gd.last_status[s] = st != 0 ? st : -5;
      }
      const double step = a.gd.eta[s] / (double)(n_s > 0 ? n_s : 1);
      for (int q = 0; q < P; ++q) th_prop[q] = pl.par_free[q] ? th_acc[q] - step * g_acc[q] : th_acc[q];
    }
  }
  if constexpr (FIT) {
    __syncthreads();
    compute_pertheta<M>(pl, a.gd.th_prop + (size_t)s * P, a.glx, a.glw, &a.consts[s], small);
  }
}

template <class M>
__global__ __launch_bounds__(kBlock) void k_fit_init(const Plan pl, const double* __restrict__ theta,
                                                    int n_sets, double eta, GDState gd,
                                                    PerTheta* __restrict__ consts,
                                                    const double* __restrict__ glx,
                                                    const double* __restrict__ glw) {
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  const int s = blockIdx.x;
  if (s >= n_sets) return;
  const int P = pl.n_param;
  if (threadIdx.x < P) {
    const double v = theta[(size_t)s * P + threadIdx.x];
    gd.th_acc[(size_t)s * P + threadIdx.x] = v;
    gd.th_prop[(size_t)s * P + threadIdx.x] = v;
    gd.g_acc[(size_t)s * P + threadIdx.x] = 0.0;
  }
  if (threadIdx.x == 0) {
    gd.f_acc[s] = __builtin_inf();
    gd.eta[s] = eta;
    gd.last_status[s] = 0;
  }
  __syncthreads();
  compute_pertheta<M>(pl, theta + (size_t)s * P, glx, glw, &consts[s], small);
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <class M>
struct Launch {
  template <bool GRAD, int U>
  static hipError_t single_u(const Plan& pl, const SingleArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_single<M, GRAD, U>), dim3(grid), dim3(kBlock), 0, st, pl, a);
    return hipGetLastError();
  }
  static hipError_t single(const Plan& pl, const SingleArgs& a, bool grad, int unroll, int grid,
                           hipStream_t st) {
    if (grad) return unroll >= 4 ? single_u<true, 4>(pl, a, grid, st) : single_u<true, 2>(pl, a, grid, st);
    return unroll >= 4 ? single_u<false, 4>(pl, a, grid, st) : single_u<false, 2>(pl, a, grid, st);
  }
  static hipError_t consts(const Plan& pl, const double* theta, int n_sets, PerTheta* out, const double* glx,
                           const double* glw, hipStream_t st) {
    hipLaunchKernelGGL((k_consts<M>), dim3(n_sets), dim3(kBlock), 0, st, pl, theta, n_sets, out, glx, glw);
    return hipGetLastError();
  }
  static hipError_t sets(const Plan& pl, const SetsArgs& a, bool grad, bool fit, int grid, hipStream_t st) {
    if (grad || fit) hipLaunchKernelGGL((k_sets<M, true, 2>), dim3(grid), dim3(kBlock), 0, st, pl, a);
    else hipLaunchKernelGGL((k_sets<M, false, 2>), dim3(grid), dim3(kBlock), 0, st, pl, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 fg(a.n_sets > 0 ? a.n_sets : 1);
    if (fit) hipLaunchKernelGGL((k_sets_finish<M, true, true>), fg, dim3(kBlock), 0, st, pl, a);
    else if (grad) hipLaunchKernelGGL((k_sets_finish<M, true, false>), fg, dim3(kBlock), 0, st, pl, a);
    else hipLaunchKernelGGL((k_sets_finish<M, false, false>), fg, dim3(kBlock), 0, st, pl, a);
    return hipGetLastError();
  }
  static hipError_t fit_init(const Plan& pl, const double* theta, int n_sets, double eta, const GDState& gd,
                             PerTheta* consts, const double* glx, const double* glw, hipStream_t st) {
    hipLaunchKernelGGL((k_fit_init<M>), dim3(n_sets), dim3(kBlock), 0, st, pl, theta, n_sets, eta, gd, consts,
                       glx, glw);
    return hipGetLastError();
  }
};

template <class M, int l = 0>
void fill_slots(VariantOps& v) {
  if constexpr (l < M::L) {
    using Sl = typename M::template S<l>;
    v.kind[l] = Sl::Leaf::kKind;
    v.obs[l] = Sl::obs;
    v.root[l] = Sl::root ? 1 : 0;
    v.np[l] = Sl::Leaf::NP;
    fill_slots<M, l + 1>(v);
  }
}

template <class M>
VariantOps make_ops(const char* name) {
  VariantOps v{};
  v.name = name;
  v.K = M::K;
  v.nobs = M::NOBS;
  v.n_leaf = M::L;
  fill_slots<M>(v);
  v.na_grad = M::NA_GRAD;
  v.single = &Launch<M>::single;
  v.consts = &Launch<M>::consts;
  v.sets = &Launch<M>::sets;
  v.fit_init = &Launch<M>::fit_init;
  return v;
}

}  // namespace nllmi
