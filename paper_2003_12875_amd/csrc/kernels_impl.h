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

// Gradient descent on the mean NLL with step halving, by a whole block:
// thread 0 accepts the evaluated proposal when its NLL is finite and exceeds
// the last accepted one by at most 4 ulps (rounding noise), else halves the
// step; then thread q forms the next proposal theta_acc - eta g_acc / N of
// parameter q (free parameters only).  st/nll/grad are valid in thread 0;
// grad is in shared memory.
__device__ inline void gd_update(const Plan& pl, const GDState& gd, int s, int st, double nll,
                                 const double* grad, int64_t n_s) {
  __shared__ int s_ok;
  __shared__ double s_step;
  const int P = pl.n_param;
  if (threadIdx.x == 0) {
    const double fa = gd.f_acc[s];
    const bool ok = st == 0 && __builtin_isfinite(nll) && nll <= fa + 4.0 * 2.220446049250313e-16 * fabs(fa);
    if (ok) {
      gd.f_acc[s] = nll;
      gd.last_status[s] = 0;
    } else {
      gd.eta[s] *= 0.5;
      if (!__builtin_isfinite(fa)) gd.last_status[s] = st != 0 ? st : -5;
    }
    s_ok = ok;
    s_step = gd.eta[s] / (double)(n_s > 0 ? n_s : 1);
  }
  __syncthreads();
  const int q = threadIdx.x;
  if (q < P) {
    double* th_acc = gd.th_acc + (size_t)s * P;
    double* g_acc = gd.g_acc + (size_t)s * P;
    double* th_prop = gd.th_prop + (size_t)s * P;
    double acc = th_acc[q], ga = g_acc[q];
    if (s_ok) {
      acc = th_prop[q];
      ga = grad[q];
      th_acc[q] = acc;
      g_acc[q] = ga;
    }
    th_prop[q] = pl.par_free[q] ? acc - s_step * ga : acc;
  }
}

// ------------------------------------------------------------------------
// per-tile event loops
// ------------------------------------------------------------------------
template <class M, int U>
__device__ inline void load_tile(const double* const* cols, int64_t base, double (&x)[U][M::NOBS]) {
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int o = 0; o < M::NOBS; ++o) x[u][o] = cols[o][base + (int64_t)u * kBlock];
}

template <class M, bool GRAD, int U>
__device__ inline void compute_tile(const double (&x)[U][M::NOBS], const Consts<M>& C, Acc<M, GRAD>& acc) {
#pragma unroll
  for (int u = 0; u < U; ++u) model_event<M, GRAD>(x[u], C, acc);
  acc.renorm();
}

// Full tiles base0, base0 + stride, ... (count of them), software
// pipelined: the first tile arrives preloaded in xn, and the loads of the
// next tile are issued before the current one is computed so that two tiles
// of loads are in flight per wave.
template <class M, bool GRAD, int U>
__device__ inline void stream_tiles(const double* const* cols, int64_t base0, int64_t stride, int64_t count,
                                    double (&xn)[U][M::NOBS], const Consts<M>& C, Acc<M, GRAD>& acc) {
  for (int64_t k = 0; k < count; ++k) {
    double xc[U][M::NOBS];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int o = 0; o < M::NOBS; ++o) xc[u][o] = xn[u][o];
    if (k + 1 < count) load_tile<M, U>(cols, base0 + (k + 1) * stride, xn);
    compute_tile<M, GRAD, U>(xc, C, acc);
  }
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
// Streaming pass over one dataset: per-block prologue, the block's tiles,
// one compensated partial per block (plain stores; the next kernel on the
// stream reads them).  Block 0 also leaves its per-point constants for the
// finishing kernel.
template <class M, bool GRAD, int U, bool FIT = false>
__global__ __launch_bounds__(kBlock) void k_single(const Plan pl, const SingleArgs a) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;  // + invalid-event count
  __shared__ PerTheta pt;
  __shared__ DD red[4 * NV];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];

  const double* cols[M::NOBS];
#pragma unroll
  for (int o = 0; o < M::NOBS; ++o) cols[o] = a.cols[o];
  const int64_t tile = (int64_t)kBlock * U;
  const int64_t nfull = a.n / tile;
  const int64_t mine = nfull > (int64_t)blockIdx.x ? (nfull - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t base0 = (int64_t)blockIdx.x * tile + threadIdx.x;
  // the first tile does not depend on theta: its loads overlap the prologue
  double xn[U][M::NOBS];
  if (mine > 0) load_tile<M, U>(cols, base0, xn);

  const double* theta = FIT ? a.gd.th_prop : a.theta;
  compute_pertheta<M>(pl, theta, a.glx, a.glw, &pt, small);
  Consts<M> C;
  C.load(pt, pl);
  Acc<M, GRAD> acc;
  acc.init();
  if (uniform(pt.bad) == 0) {
    stream_tiles<M, GRAD, U>(cols, base0, (int64_t)gridDim.x * tile, mine, xn, C, acc);
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
  if (threadIdx.x < NV) reinterpret_cast<DD*>(a.partials)[(size_t)blockIdx.x * NV + threadIdx.x] = tot[threadIdx.x];
  if (blockIdx.x == 0) {
    const double* src = reinterpret_cast<const double*>(&pt);
    double* dst = reinterpret_cast<double*>(a.pt_out);
    for (int i = threadIdx.x; i < (int)(sizeof(PerTheta) / sizeof(double)); i += kBlock) dst[i] = src[i];
  }
}

// Finishing kernel (one block of kFinishBlock threads): the block partials
// in block order, then NLL and gradient; in fit mode the gradient-descent
// step of the proposal just evaluated.
template <class M, bool GRAD, bool FIT = false>
__global__ __launch_bounds__(kFinishBlock) void k_single_finish(const Plan pl, const SingleArgs a, int n_blocks) {
  constexpr int NA = M::template NA<GRAD>;
  constexpr int NV = NA + 1;
  __shared__ DD red[kFinishBlock];
  __shared__ DD tot[NV];
  __shared__ double s_grad[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_nll;
  __shared__ int s_st;
  {  // one parallel copy of the per-point constants and theta
    const double* src = reinterpret_cast<const double*>(a.pt_out);
    double* dst = reinterpret_cast<double*>(&spt);
    for (int i = threadIdx.x; i < (int)(sizeof(PerTheta) / sizeof(double)); i += kFinishBlock) dst[i] = src[i];
    const double* th = FIT ? a.gd.th_prop : a.theta;
    if (threadIdx.x < pl.n_param) s_theta[threadIdx.x] = th[threadIdx.x];
  }
  sum_records<NV, kFinishBlock>(reinterpret_cast<const DD*>(a.partials), n_blocks, red, tot);
  if (threadIdx.x == 0) {
    s_st = finish<M, GRAD>(pl, spt, tot, (int64_t)(tot[NA].hi + tot[NA].lo), a.n, s_theta, &s_nll, s_grad);
  }
  __syncthreads();
  if constexpr (FIT) {
    gd_update(pl, a.gd, 0, s_st, s_nll, s_grad, a.n);
  } else {
    if (threadIdx.x == 0) {
      *a.nll_out = s_nll;
      if (s_st == -3) atomicOr(a.status, (int)kStatusParam);
      if (s_st == -5) atomicOr(a.status, (int)kStatusPdf);
    }
    if (GRAD && a.grad_out && threadIdx.x < pl.n_param) a.grad_out[threadIdx.x] = s_grad[threadIdx.x];
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
      const int64_t full = (end - start) / step;
      double xn[U][M::NOBS];
      if (full > 0) load_tile<M, U>(cols, start + threadIdx.x, xn);
      stream_tiles<M, GRAD, U>(cols, start + threadIdx.x, step, full, xn, C, acc);
      const int64_t base = start + full * step;
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
  __shared__ DD red[kBlock];
  __shared__ DD tot[NV];
  __shared__ double small[4 * (kMaxLeafParams + 1)];
  __shared__ double s_grad[kMaxParams];
  __shared__ PerTheta spt;
  __shared__ double s_theta[kMaxParams];
  __shared__ double s_nll;
  __shared__ int s_st;
  const int s = blockIdx.x;
  if (s >= a.n_sets) return;
  const int P = pl.n_param;
  {  // one parallel copy of the set's constants and parameters
    const double* src = reinterpret_cast<const double*>(&a.consts[s]);
    double* dst = reinterpret_cast<double*>(&spt);
    for (int i = threadIdx.x; i < (int)(sizeof(PerTheta) / sizeof(double)); i += kBlock) dst[i] = src[i];
    const double* th = FIT ? a.gd.th_prop + (size_t)s * P : a.theta + (size_t)s * P;
    if (threadIdx.x < P) s_theta[threadIdx.x] = th[threadIdx.x];
  }
  const int64_t first = a.tile_off[s], n_items = a.tile_off[s + 1] - first;
  sum_records<NV, kBlock>(reinterpret_cast<const DD*>(a.partials) + (size_t)first * NV, n_items, red, tot);
  const int flag = a.set_flag[s];
  const int64_t n_s = flag ? 0 : a.offsets[s + 1] - a.offsets[s];
  if (threadIdx.x == 0) {
    double nll;
    int st = finish<M, GRAD>(pl, spt, tot, (int64_t)(tot[NA].hi + tot[NA].lo), n_s, s_theta, &nll, s_grad);
    if (flag) {
      st = -1;
      nll = __builtin_inf();
    }
    s_st = st;
    s_nll = nll;
  }
  __syncthreads();
  if constexpr (!FIT) {
    if (threadIdx.x == 0) {
      a.nll_out[s] = s_nll;
      if (a.status_out) a.status_out[s] = s_st;
    }
    if (GRAD && a.grad_out && threadIdx.x < P)
      a.grad_out[(size_t)s * P + threadIdx.x] = s_st == 0 ? s_grad[threadIdx.x] : 0.0;
  } else {
    gd_update(pl, a.gd, s, s_st, s_nll, s_grad, n_s);
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
  template <bool GRAD, bool FIT>
  static hipError_t single_t(const Plan& pl, const SingleArgs& a, int unroll, int grid, hipStream_t st) {
    if (unroll >= 4) hipLaunchKernelGGL((k_single<M, GRAD, 4, FIT>), dim3(grid), dim3(kBlock), 0, st, pl, a);
    else hipLaunchKernelGGL((k_single<M, GRAD, 2, FIT>), dim3(grid), dim3(kBlock), 0, st, pl, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_single_finish<M, GRAD, FIT>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
    return hipGetLastError();
  }
  static hipError_t single_fit(const Plan& pl, const SingleArgs& a, int unroll, int grid, hipStream_t st) {
    return single_t<true, true>(pl, a, unroll, grid, st);
  }
  static hipError_t single(const Plan& pl, const SingleArgs& a, bool grad, int unroll, int grid,
                           hipStream_t st) {
    return grad ? single_t<true, false>(pl, a, unroll, grid, st) : single_t<false, false>(pl, a, unroll, grid, st);
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
  v.single_fit = &Launch<M>::single_fit;
  v.consts = &Launch<M>::consts;
  v.sets = &Launch<M>::sets;
  v.fit_init = &Launch<M>::fit_init;
  return v;
}

}  // namespace nllmi
