// kernels_impl.h -- launchers of the streaming NLL kernels and the
// registry entry of a compiled model shape (instantiated per shape in
// variants_*.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "kernels_dev.h"

namespace nllmi {

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
// dynamic LDS that pads a block of `kernel` to lds_cap bytes (0: no cap)
inline size_t pad_lds(const void* kernel, int lds_cap) {
  if (lds_cap <= 0) return 0;
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) return 0;
  return (size_t)lds_cap > fa.sharedSizeBytes ? (size_t)lds_cap - fa.sharedSizeBytes : 0;
}

template <class M>
struct Launch {
  // events per thread per tile compiled for this shape: {2, 4, 8}, or
  // {2, 4} for weighted shapes and shapes with more than 8 accumulators
  // (registers); 8 maps to 4 there
  static constexpr bool kU8 = !M::WEIGHTED && M::NA_GRAD <= 8;
  static int pick_u(int unroll) { return unroll >= 8 && kU8 ? 8 : unroll >= 4 ? 4 : 2; }

  // With timing events (ev0, ev1 both set) the launch carries them, so that
  // they record the dispatch's own start and end (as a profiler's kernel
  // trace does) rather than bracketing it with the queue's gaps.
  template <bool GRAD, bool FIT, int U>
  static void launch_single(const Plan& pl, const SingleArgs& a, int grid, int lds_cap, hipStream_t st,
                            hipEvent_t ev0, hipEvent_t ev1) {
    const void* k = reinterpret_cast<const void*>(&k_single<M, GRAD, U, FIT>);
    if (ev0 && ev1)
      hipExtLaunchKernelGGL((k_single<M, GRAD, U, FIT>), dim3(grid), dim3(kBlock), (uint32_t)pad_lds(k, lds_cap), st,
                            ev0, ev1, 0u, pl, a);
    else
      hipLaunchKernelGGL((k_single<M, GRAD, U, FIT>), dim3(grid), dim3(kBlock), pad_lds(k, lds_cap), st, pl, a);
  }
  template <bool GRAD, bool FIT>
  static hipError_t single_t(const Plan& pl, const SingleArgs& a, int unroll, int grid, int lds_cap, hipStream_t st,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    const int u = pick_u(unroll);
    if constexpr (kU8) {
      if (u == 8) launch_single<GRAD, FIT, 8>(pl, a, grid, lds_cap, st, ev0, ev1);
    }
    if (u == 4) launch_single<GRAD, FIT, 4>(pl, a, grid, lds_cap, st, ev0, ev1);
    if (u == 2) launch_single<GRAD, FIT, 2>(pl, a, grid, lds_cap, st, ev0, ev1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_single_finish<M, GRAD, FIT>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
    return hipGetLastError();
  }
  template <int U>
  static void launch_fit(const Plan& pl, const SingleArgs& a, int grid, int lds_cap, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1) {
    const void* k = reinterpret_cast<const void*>(&k_single_fit<M, U>);
    if (ev0 && ev1)
      hipExtLaunchKernelGGL((k_single_fit<M, U>), dim3(grid), dim3(kBlock), (uint32_t)pad_lds(k, lds_cap), st, ev0,
                            ev1, 0u, pl, a);
    else
      hipLaunchKernelGGL((k_single_fit<M, U>), dim3(grid), dim3(kBlock), pad_lds(k, lds_cap), st, pl, a);
  }
  // one gradient-descent step (k_single_fit: the previous step's update,
  // then this step's pass)
  static hipError_t single_fit(const VariantOps&, const Plan& pl, const SingleArgs& a, int unroll, int grid, int lds_cap, hipStream_t st,
                               hipEvent_t ev0, hipEvent_t ev1) {
    const int u = pick_u(unroll);
    if constexpr (kU8) {
      if (u == 8) launch_fit<8>(pl, a, grid, lds_cap, st, ev0, ev1);
    }
    if (u == 4) launch_fit<4>(pl, a, grid, lds_cap, st, ev0, ev1);
    if (u == 2) launch_fit<2>(pl, a, grid, lds_cap, st, ev0, ev1);
    return hipGetLastError();
  }
  // the update of the last step's proposal (grid: that launch's blocks)
  static hipError_t fit_finish(const VariantOps&, const Plan& pl, const SingleArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_single_finish<M, true, true>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
    return hipGetLastError();
  }
  // BHHH: compiled for FP64 shapes with at most 6 score features (21 second
  // moments), at 2 and 4 events per thread per tile (8 maps to 4)
  static constexpr bool kBH = bh_compiled<M>();
  template <bool FIT, int U>
  static void launch_bh(const Plan& pl, const SingleArgs& a, int grid, int lds_cap, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
    const void* k = reinterpret_cast<const void*>(&k_single<M, true, U, FIT, true>);
    if (ev0 && ev1)
      hipExtLaunchKernelGGL((k_single<M, true, U, FIT, true>), dim3(grid), dim3(kBlock), (uint32_t)pad_lds(k, lds_cap),
                            st, ev0, ev1, 0u, pl, a);
    else
      hipLaunchKernelGGL((k_single<M, true, U, FIT, true>), dim3(grid), dim3(kBlock), pad_lds(k, lds_cap), st, pl, a);
  }
  template <bool FIT>
  static hipError_t bh_t(const Plan& pl, const SingleArgs& a, int unroll, int grid, int lds_cap, hipStream_t st,
                         hipEvent_t ev0, hipEvent_t ev1) {
    if constexpr (kBH) {
      if (unroll >= 4) launch_bh<FIT, 4>(pl, a, grid, lds_cap, st, ev0, ev1);
      else launch_bh<FIT, 2>(pl, a, grid, lds_cap, st, ev0, ev1);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_single_finish<M, true, FIT, true>), dim3(1), dim3(kFinishBlock), 0, st, pl, a, grid);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static hipError_t single_bhhh(const VariantOps&, const Plan& pl, const SingleArgs& a, int unroll, int grid, int lds_cap,
                                hipStream_t st) {
    return bh_t<false>(pl, a, unroll, grid, lds_cap, st, nullptr, nullptr);
  }
  static hipError_t single_bhhh_fit(const VariantOps&, const Plan& pl, const SingleArgs& a, int unroll, int grid, int lds_cap,
                                    hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    return bh_t<true>(pl, a, unroll, grid, lds_cap, st, ev0, ev1);
  }
  static hipError_t single(const VariantOps&, const Plan& pl, const SingleArgs& a, bool grad, int unroll, int grid, int lds_cap,
                           hipStream_t st) {
    return grad ? single_t<true, false>(pl, a, unroll, grid, lds_cap, st)
                : single_t<false, false>(pl, a, unroll, grid, lds_cap, st);
  }
  static hipError_t consts(const VariantOps&, const Plan& pl, const double* theta, int n_sets, PerTheta* out, double* aux,
                           const double* glx, const double* glw, hipStream_t st) {
    hipLaunchKernelGGL((k_consts<M>), dim3(n_sets), dim3(kBlock), 0, st, pl, theta, n_sets, out, aux, glx, glw);
    return hipGetLastError();
  }
  template <bool GRAD, int U>
  static void launch_sets(const Plan& pl, const SetsArgs& a, int grid, int lds_cap, hipStream_t st, hipEvent_t ev0,
                          hipEvent_t ev1) {
    const void* k = reinterpret_cast<const void*>(&k_sets<M, GRAD, U>);
    if (ev0 && ev1)
      hipExtLaunchKernelGGL((k_sets<M, GRAD, U>), dim3(grid), dim3(kBlock), (uint32_t)pad_lds(k, lds_cap), st, ev0,
                            ev1, 0u, pl, a, static_cast<const WorkItem*>(a.items),
                            static_cast<const PerTheta*>(a.consts), a.chunk_first);
    else
      hipLaunchKernelGGL((k_sets<M, GRAD, U>), dim3(grid), dim3(kBlock), pad_lds(k, lds_cap), st, pl, a,
                         static_cast<const WorkItem*>(a.items), static_cast<const PerTheta*>(a.consts),
                         a.chunk_first);
  }
  template <bool GRAD>
  static void sets_u(const Plan& pl, const SetsArgs& a, int unroll, int grid, int lds_cap, hipStream_t st,
                     hipEvent_t ev0, hipEvent_t ev1) {
    const int u = pick_u(unroll);
    if constexpr (kU8) {
      if (u == 8) launch_sets<GRAD, 8>(pl, a, grid, lds_cap, st, ev0, ev1);
    }
    if (u == 4) launch_sets<GRAD, 4>(pl, a, grid, lds_cap, st, ev0, ev1);
    if (u == 2) launch_sets<GRAD, 2>(pl, a, grid, lds_cap, st, ev0, ev1);
  }
  static hipError_t sets(const VariantOps&, const Plan& pl, const SetsArgs& a, bool grad, bool fit, int unroll, int grid, int lds_cap,
                         hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (a.n_sets <= 0) return hipSuccess;  // the finishing kernel's grid is one block per set
    if (grad || fit) sets_u<true>(pl, a, unroll, grid, lds_cap, st, ev0, ev1);
    else sets_u<false>(pl, a, unroll, grid, lds_cap, st, ev0, ev1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 fg(a.n_sets), fb(finish_threads<M>());
    if (fit) hipLaunchKernelGGL((k_sets_finish<M, true, true>), fg, fb, 0, st, pl, a);
    else if (grad) hipLaunchKernelGGL((k_sets_finish<M, true, false>), fg, fb, 0, st, pl, a);
    else hipLaunchKernelGGL((k_sets_finish<M, false, false>), fg, fb, 0, st, pl, a);
    return hipGetLastError();
  }
  static hipError_t fit_init(const VariantOps&, const Plan& pl, const double* theta, int n_sets, double eta, const GDState& gd,
                             PerTheta* consts, double* aux, const double* glx, const double* glw, hipStream_t st) {
    hipLaunchKernelGGL((k_fit_init<M>), dim3(n_sets), dim3(kBlock), 0, st, pl, theta, n_sets, eta, gd, consts, aux,
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
  v.na_grad = M::template NA<true>;  // accumulators per record (counters included)
  v.precision = M::PREC;
  v.flat = M::FLAT ? 1 : 0;
  v.aux = M::AUX ? 1 : 0;
  v.fin_threads = finish_threads<M>();
  v.rtc = nullptr;
  v.single = &Launch<M>::single;
  v.single_fit = &Launch<M>::single_fit;
  v.fit_finish = &Launch<M>::fit_finish;
  v.consts = &Launch<M>::consts;
  v.sets = &Launch<M>::sets;
  v.fit_init = &Launch<M>::fit_init;
  if constexpr (M::PREC == 0 && M::NOBS < kMaxObs) {  // weighted events: the weights take one column
    v.single_w = &Launch<Weighted<M>>::single;
    v.single_w_fit = &Launch<Weighted<M>>::single_fit;
    v.w_fit_finish = &Launch<Weighted<M>>::fit_finish;
  }
  if constexpr (Launch<M>::kBH) {
    v.single_bhhh = &Launch<M>::single_bhhh;
    v.single_bhhh_fit = &Launch<M>::single_bhhh_fit;
    v.bhhh_record = M::template NA<true> + 1 + AccBhhh<M>::NM;
  }
  return v;
}

}  // namespace nllmi
