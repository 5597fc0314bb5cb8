// model.h -- compile-time model shapes, the fused per-event pass and the
// per-parameter-point prologue.
//
// A compiled model is Model<K, NOBS, Slot<Leaf, obs, root>...>: the leaf
// types, the observable each reads and whether it is a factor of every
// term are template parameters, so the per-event work is straight-line
// code; which non-root leaf belongs to which of the K terms and the term
// weights are runtime (uniform) data in the Plan.
//
// Per event (Sec. 5.1: one expression per dataset entry; Sec. 5.3: no data
// dependence between entries, intermediates kept in registers):
//   lam_l, gam_l, phi_l       from every leaf
//   L_k = ck_k + sum_{l in S_k, not root} lam_l
//   log p = croot + sum_{root l} (lam_l + log gam_l) + logsumexp_k L_k
// The log-sum-exp is split as m = max_k L_k (summed) and s = sum_k
// e^{L_k - m} in [1, K] (multiplied into a running mantissa/exponent
// product whose log is taken once per thread), so a K = 2 mixture costs one
// exp and no log per event, and a single-term model (e.g. one Gaussian)
// costs no transcendental at all.
// Gradient (the adjoint of that expression):
//   d log p / d theta = sum_k r_k dC_k + sum_l R_l fscale_lp phi_lp,
//   r_k = e^{L_k - m} / s,  R_l = sum_{k contains l} r_k  (1 for root leaves)
// and the parameter-only parts (dC_k, fscale, d log Z) are applied once,
// after the reduction, to the accumulated sums of r_k and R_l phi_lp
// (the sum of r_{K-1} is N minus the others: sum_k r_k = 1 per event).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include <tuple>
#include <type_traits>
#include <utility>

#include "fp32.h"
#include "fp64.h"
#include "leaves.h"
#include "plan.h"

namespace nllmi {

template <class F, int... I>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// broadcast lane 0's value: the compiler then keeps it in scalar registers
__device__ inline double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class LeafT, int OBS, bool ROOT>
struct Slot {
  using Leaf = LeafT;
  static constexpr int obs = OBS;
  static constexpr bool root = ROOT;
  static constexpr bool lin = ROOT && LeafT::kLinear;  // linear factor, no per-event log
  // linear factor of its term: the term contributes e_k * gamma to the sum
  // s whose log is taken once per thread, so no per-event log either
  static constexpr bool tlin = !ROOT && LeafT::kLinear;
};

template <int K_, int NOBS_, class... Slots>
struct Model {
  static constexpr int K = K_;
  static constexpr int NOBS = NOBS_;
  static constexpr int L = sizeof...(Slots);
  using SlotTuple = std::tuple<Slots...>;
  template <int l>
  using S = std::tuple_element_t<l, SlotTuple>;

  static constexpr int NPT = (Slots::Leaf::NP + ... + 0);
  static constexpr bool HAS_LIN = (Slots::lin || ...);
  static constexpr bool HAS_TLIN = (Slots::tlin || ...);
  static constexpr bool NEED_PROD = (K > 1) || HAS_LIN;
  static constexpr int TERM_BASE = 1;
  static constexpr int LEAF_BASE = 1 + (K > 1 ? K : 0);
  static constexpr int NA_GRAD = LEAF_BASE + NPT;
  template <bool GRAD>
  static constexpr int NA = GRAD ? NA_GRAD : 1;

  static constexpr int NPs[L] = {Slots::Leaf::NP...};
  static constexpr bool ROOTs[L] = {Slots::root...};
  static constexpr int NR = ((Slots::root ? 0 : 1) + ... + 0);  // non-root leaves
  static constexpr bool HAS_ROOT = NR < L;
  // Flat mixture: term k consists of the k-th non-root leaf (and the root
  // factors); the host orders the terms accordingly.
  static constexpr bool FLAT = K > 1 && NR == K;
  template <int l>
  static constexpr int term_of() {  // term of non-root leaf l (flat shapes)
    int k = 0;
    for (int i = 0; i < l; ++i) k += ROOTs[i] ? 0 : 1;
    return k;
  }
  template <int l>
  static constexpr int leaf_off() {
    int o = 0;
    for (int i = 0; i < l; ++i) o += NPs[i];
    return o;
  }
  using LeafCs = std::tuple<typename Slots::Leaf::C...>;
  using LeafC32s = std::tuple<typename Slots::Leaf::C32...>;
  static constexpr int PREC = 0;  // 0: FP64 event pass, 1: FP32-compensated
  static constexpr bool WEIGHTED = false;
  // a logarithm per event (the kernels stage g_log_tab)
  static constexpr bool EVENT_LOG = (Slots::Leaf::kEventLog || ...);
  // a leaf with per-point tables beside PerTheta (at most one)
  static constexpr bool AUX = (Slots::Leaf::kAux || ...);
  static_assert(((Slots::Leaf::kAux ? 1 : 0) + ... + 0) <= 1, "at most one leaf with per-point tables");

  static_assert(L >= 1 && L <= kMaxLeaves, "1..kMaxLeaves leaves");
  static_assert(K >= 1 && K <= kMaxTerms, "1..kMaxTerms terms");
  static_assert(NA_GRAD <= kMaxAcc, "accumulator budget");
};

// A shape with as many non-root leaves as terms whose terms are not one
// non-root leaf each (a product of two sums: (a + b)(c + d) has four terms
// of two non-root leaves): the plan's term masks define the terms.
template <class B>
struct NonFlat : B {
  static constexpr bool FLAT = false;
};

// The same compiled shape with the FP32-compensated event pass.  Its sums
// gain K - 1 counters: how many events have term k (k >= 1) as the largest
// one, so that the constant ck_k - ck_0 of that term is added count_k times
// in FP64 instead of being rounded into every event's FP32 value.
template <class Base>
struct FP32C : Base {
  static_assert(!Base::AUX, "no FP32-compensated pass for leaves with per-point tables");
  static constexpr int PREC = 1;
  static constexpr bool EVENT_LOG = false;  // single-precision logarithms of its own
  static constexpr int NCNT = Base::K > 1 ? Base::K - 1 : 0;
  template <bool GRAD>
  static constexpr int CNT_BASE = Base::template NA<GRAD>;
  template <bool GRAD>
  static constexpr int NA = Base::template NA<GRAD> + NCNT;
  static_assert(Base::NA_GRAD + NCNT <= kMaxAcc, "accumulator budget");
};

// The same compiled shape over weighted events (a binned dataset as its bin
// centres weighted by the counts, or sWeighted events; Sec. 5.1 sets such
// binned fits against unbinned ones): the weights are one more column,
// read after the observables.  Each event's log-density and gradient
// features enter the sums multiplied by its weight.  After the reduction
// the weights' sum W (computed once when the weights are attached, so that
// it does not depend on the parameter point) takes the place of the event
// count N: in the term constants, the last term's responsibility total, the
// root leaves' normalisation terms, the extended term nu - W ln nu and the
// gradient-descent scale 1/W.
template <class B>
struct Weighted : B {
  using Base = B;
  static constexpr bool WEIGHTED = true;
  static constexpr bool EVENT_LOG = true;  // each event's log-density
  static constexpr int NOBS = B::NOBS + 1;
  static_assert(B::PREC == 0 && !B::WEIGHTED, "weighted events: FP64 event pass");
  static_assert(NOBS <= kMaxObs, "weights take one observable slot");
};

// Uniform per-point constants of a compiled model, held in scalar registers.
template <class M>
struct Consts {
  // mixtures take one e^x per event from the LDS table of exp_nonpos_tab;
  // the kernel stages it and sets etab
  static constexpr bool kExpTab = M::K > 1;
  typename M::LeafCs leaf;
  double ck[M::K];
  int mask[M::K];  // non-root leaves of term k
  const double* etab;

  // aux: the per-point tables of a leaf that has them (else unused)
  __device__ void load(const PerTheta& pt, const Plan& pl, const double* aux) {
    static_for<M::L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      using Leaf = typename M::template S<l>::Leaf;
      if constexpr (Leaf::kAux) {
        std::get<l>(leaf) = Leaf::load_aux(aux);
      } else {
        double ec[kLeafConsts];
#pragma unroll
        for (int j = 0; j < kLeafConsts; ++j) ec[j] = uniform(pt.ec[l][j]);
        std::get<l>(leaf) = Leaf::load(ec);
      }
    });
#pragma unroll
    for (int k = 0; k < M::K; ++k) {
      ck[k] = uniform(pt.ck[k]);
      mask[k] = uniform(pl.term_mask[k]);
    }
  }
};

template <class M, bool GRAD>
struct Acc {
  static constexpr int NA = M::template NA<GRAD>;
  double a[M::template NA<GRAD>];
  double P;    // running product (mantissa)
  int E;       // its binary exponent
  int bad;     // events with p <= 0 or non-finite
  __device__ void init() {
#pragma unroll
    for (int j = 0; j < M::template NA<GRAD>; ++j) a[j] = 0.0;
    P = 1.0;
    E = 0;
    bad = 0;
  }
  __device__ void renorm() {
    if constexpr (M::NEED_PROD) {
      int e;
      P = frexp(P, &e);
      E += e;
    }
  }
  __device__ void begin_tile() {}
  __device__ void end_tile() { renorm(); }
  // fold the product into the log-sum and hand out the thread's sums
  __device__ void finalize(double (&v)[NA]) {
    if constexpr (M::NEED_PROD) a[0] += log(P) + (double)E * kLn2;
#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = a[j];
  }
};

template <class M, bool GRAD>
__device__ inline void model_event(const double (&x)[M::NOBS], const Consts<M>& C, Acc<M, GRAD>& acc) {
  constexpr int L = M::L, K = M::K;
  double lam[L];
  double gl[L];  // linear factors of term leaves
  double gprod = 1.0;
  double phi[M::NPT > 0 ? M::NPT : 1];
  static_for<L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    using Sl = typename M::template S<l>;
    double gam;
    if constexpr (Sl::Leaf::kLinear) {
      Sl::Leaf::template event<GRAD, Sl::lin || Sl::tlin>(x[Sl::obs], std::get<l>(C.leaf), lam[l], gam,
                                                           &phi[M::template leaf_off<l>()]);
    } else {
      Sl::Leaf::template event<GRAD>(x[Sl::obs], std::get<l>(C.leaf), lam[l], gam,
                                     &phi[M::template leaf_off<l>()]);
    }
    if constexpr (Sl::lin) gprod *= gam;
    if constexpr (Sl::tlin) {
      gl[l] = gam;
      acc.bad += !(gam >= 0.0);  // a negative linear term is an invalid density
    } else {
      gl[l] = 1.0;
    }
  });

  double rootsum = 0.0;
  if constexpr (M::HAS_ROOT) {
    bool first = true;
    static_for<L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      if constexpr (M::template S<l>::root) {
        rootsum = first ? lam[l] : rootsum + lam[l];
        first = false;
      }
    });
  }

  if constexpr (K == 1) {
    acc.a[0] += rootsum;
    // a non-finite log value propagates into the sum by itself; only the sign
    // of a linear factor has to be checked (two negative factors would cancel)
    if constexpr (M::HAS_LIN) {
      acc.P *= gprod;
      acc.bad += !(gprod > 0.0);
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int j = 0; j < M::NPT; ++j) acc.a[M::LEAF_BASE + j] += phi[j];
    }
  } else {
    double Lk[K];
    double Gk[K];  // term linear factors (1 without linear term leaves)
    if constexpr (M::FLAT) {
      static_for<L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if constexpr (!M::template S<l>::root) {
          Lk[M::template term_of<l>()] = C.ck[M::template term_of<l>()] + lam[l];
          Gk[M::template term_of<l>()] = gl[l];
        }
      });
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double v = C.ck[k], g = 1.0;
        static_for<L>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          if constexpr (!M::template S<l>::root) {
            const bool in = (C.mask[k] >> l) & 1;
            v += in ? lam[l] : 0.0;
            if constexpr (M::template S<l>::tlin) g *= in ? gl[l] : 1.0;
          }
        });
        Lk[k] = v;
        Gk[k] = g;
      }
    }
    double m, s, e[K];
    double d2 = 0.0, es2 = 0.0;  // two terms: their difference and e^-|d|
    if constexpr (K == 2) {
      const double d = Lk[0] - Lk[1];
      m = fmax(Lk[0], Lk[1]);
      const double es = exp_nonpos_tab(-fabs(d), C.etab);
      d2 = d;
      es2 = es;
      e[0] = d >= 0.0 ? 1.0 : es;
      e[1] = d >= 0.0 ? es : 1.0;
      if constexpr (M::HAS_TLIN) {
        e[0] *= Gk[0];
        e[1] *= Gk[1];
        s = e[0] + e[1];
      } else {
        s = 1.0 + es;
      }
    } else {
      m = Lk[0];
#pragma unroll
      for (int k = 1; k < K; ++k) m = fmax(m, Lk[k]);
      s = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        e[k] = exp_nonpos_tab(Lk[k] - m, C.etab);
        if constexpr (M::HAS_TLIN) e[k] *= Gk[k];
        s += e[k];
      }
    }
    double tot = m;
    if constexpr (M::HAS_ROOT) tot = rootsum + m;
    acc.a[0] += tot;
    if constexpr (M::HAS_LIN) {
      acc.P *= s * gprod;
      acc.bad += !(gprod > 0.0);
    } else {
      acc.P *= s;
    }
    if constexpr (GRAD) {
      const double inv = rcp_grad(s);  // responsibilities: gradient only
      double r[K];
      if constexpr (K == 2 && !M::HAS_TLIN) {
        // r_0 by one select; r_1 = 1 - r_0 (absolute error ~2^-48 where
        // r_1 is tiny, far below the gradient's rounding scale)
        r[0] = d2 >= 0.0 ? inv : es2 * inv;
        r[1] = 1.0 - r[0];
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) r[k] = e[k] * inv;
      }
      // the responsibilities of an event sum to 1: the last term's total is
      // N minus the others (formed after the reduction)
#pragma unroll
      for (int k = 0; k < K - 1; ++k) acc.a[M::TERM_BASE + k] += r[k];
      static_for<L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        using Sl = typename M::template S<l>;
        constexpr int off = M::template leaf_off<l>();
        if constexpr (Sl::root) {
#pragma unroll
          for (int p = 0; p < Sl::Leaf::NP; ++p) acc.a[M::LEAF_BASE + off + p] += phi[off + p];
        } else {
          double R = 0.0;
          if constexpr (M::FLAT) {
            R = r[M::template term_of<l>()];
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) R += ((C.mask[k] >> l) & 1) ? r[k] : 0.0;
          }
#pragma unroll
          for (int p = 0; p < Sl::Leaf::NP; ++p) acc.a[M::LEAF_BASE + off + p] = fma(R, phi[off + p], acc.a[M::LEAF_BASE + off + p]);
        }
      });
    }
  }
}

// ------------------------------------------------------------------------
// FP32-compensated event pass.  Per event, every observable is
// location-subtracted in FP64 and converted once; the leaves, the
// transcendental functions and the adjoint run in FP32.  A per-event FP32
// error only cancels in the sum over events if it is an unbiased rounding,
// and a per-point constant added to an FP32 value of comparable size always
// loses the same low bits (a bias that grows with N).  So every step that
// adds such a constant runs in FP64 (at the same vector rate as FP32 here)
// and is rounded to FP32 only afterwards, and products with constants use
// split constants inside an FMA.  The log-sum-exp is taken relative to
// term 0:
//   log p = croot + ck_0 + (ck_{k*} - ck_0) + [sum_root lam + L'_{k*}] + log s,
//   A_k = L'_k + (ck_k - ck_0) (FP64),  k* = argmax_k A_k,
//   s = sum_k e^{A_k - A_{k*}}
// (L'_k: the term's log-density without constants); croot + ck_0 are added
// N times and ck_k - ck_0 count_k times (count_k: events with k* = k) in
// FP64 after the reduction, so that no FP32 value carries a constant.  The per-event values are summed per tile in FP32
// and added to a per-thread (hi, lo) pair by TwoSum; the pair is widened to
// FP64 at the end.
// ------------------------------------------------------------------------
__device__ inline float uniformf(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <class M>
struct Consts32 {
  static constexpr bool kExpTab = false;
  const double* etab;
  typename M::LeafC32s leaf;
  double dck[M::K];  // ck_k - ck_0
  int mask[M::K];

  __device__ void load(const PerTheta& pt, const Plan& pl, const double* = nullptr) {
    static_for<M::L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      double ec[kLeafConsts];
#pragma unroll
      for (int j = 0; j < kLeafConsts; ++j) ec[j] = uniform(pt.ec[l][j]);
      std::get<l>(leaf) = M::template S<l>::Leaf::load32(ec);
    });
    const double c0 = uniform(pt.ck[0]);
#pragma unroll
    for (int k = 0; k < M::K; ++k) {
      dck[k] = uniform(pt.ck[k]) - c0;
      mask[k] = uniform(pl.term_mask[k]);
    }
  }
};

template <class M, bool GRAD>
struct Acc32 {
  static constexpr int NA = M::template NA<GRAD>;
  float t[NA];            // sums of the current tile
  float hi[NA], lo[NA];   // compensated per-thread sums
  float P;                // running product (mantissa)
  int E;
  int bad;
  __device__ void init() {
#pragma unroll
    for (int j = 0; j < NA; ++j) t[j] = hi[j] = lo[j] = 0.0f;
    P = 1.0f;
    E = 0;
    bad = 0;
  }
  __device__ void begin_tile() {
#pragma unroll
    for (int j = 0; j < NA; ++j) t[j] = 0.0f;
  }
  __device__ void end_tile() {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      float sum, err;
      two_sum(hi[j], t[j], sum, err);
      hi[j] = sum;
      lo[j] += err;
    }
    if constexpr (M::NEED_PROD) {
      E += __builtin_amdgcn_frexp_expf(P);
      P = __builtin_amdgcn_frexp_mantf(P);
    }
  }
  __device__ void finalize(double (&v)[NA]) {
#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = (double)hi[j] + (double)lo[j];
    if constexpr (M::NEED_PROD) v[0] += log((double)P) + (double)E * kLn2;
  }
};

template <class M, bool GRAD>
__device__ inline void model_event(const double (&x)[M::NOBS], const Consts32<M>& C, Acc32<M, GRAD>& acc) {
  constexpr int L = M::L, K = M::K;
  float lam[L];
  float gprod = 1.0f;
  float phi[M::NPT > 0 ? M::NPT : 1];
  float gl[L];
  static_for<L>([&](auto lc) {
    constexpr int l = decltype(lc)::value;
    using Sl = typename M::template S<l>;
    float gam;
    if constexpr (Sl::Leaf::kLinear) {
      Sl::Leaf::template event32<GRAD, Sl::lin || Sl::tlin>(x[Sl::obs], std::get<l>(C.leaf), lam[l], gam,
                                                             &phi[M::template leaf_off<l>()]);
    } else {
      Sl::Leaf::template event32<GRAD>(x[Sl::obs], std::get<l>(C.leaf), lam[l], gam,
                                       &phi[M::template leaf_off<l>()]);
    }
    if constexpr (Sl::lin) gprod *= gam;
    if constexpr (Sl::tlin) {
      gl[l] = gam;
      acc.bad += !(gam >= 0.0f);
    } else {
      gl[l] = 1.0f;
    }
  });

  float rootsum = 0.0f;
  if constexpr (M::HAS_ROOT) {
    bool first = true;
    static_for<L>([&](auto lc) {
      constexpr int l = decltype(lc)::value;
      if constexpr (M::template S<l>::root) {
        rootsum = first ? lam[l] : rootsum + lam[l];
        first = false;
      }
    });
  }

  if constexpr (K == 1) {
    acc.t[0] += rootsum;
    if constexpr (M::HAS_LIN) {
      acc.P *= gprod;
      acc.bad += !(gprod > 0.0f);
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int j = 0; j < M::NPT; ++j) acc.t[M::LEAF_BASE + j] += phi[j];
    }
  } else {
    float Lk[K];
    float Gk[K];
    if constexpr (M::FLAT) {
      static_for<L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        if constexpr (!M::template S<l>::root) {
          Lk[M::template term_of<l>()] = lam[l];
          Gk[M::template term_of<l>()] = gl[l];
        }
      });
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float v = 0.0f, g = 1.0f;
        static_for<L>([&](auto lc) {
          constexpr int l = decltype(lc)::value;
          if constexpr (!M::template S<l>::root) {
            const bool in = (C.mask[k] >> l) & 1;
            v += in ? lam[l] : 0.0f;
            if constexpr (M::template S<l>::tlin) g *= in ? gl[l] : 1.0f;
          }
        });
        Lk[k] = v;
        Gk[k] = g;
      }
    }
    // term log-densities relative to term 0's constant, in FP64:
    // A_k = L'_k + (ck_k - ck_0), M = A_{k*} = max_k A_k, e_k = e^{A_k - M};
    // e^a for an FP64 argument a as e^{float(a)} (1 + (a - float(a)))
    auto exp_arg = [](double a) {
      if (a < -104.0) return 0.0f;
      const float af = (float)a;
      const float e = exp_f32(af);
      return fmaf(e, (float)(a - (double)af), e);
    };
    constexpr int CB = M::template CNT_BASE<GRAD>;
    double A[K];
#pragma unroll
    for (int k = 0; k < K; ++k) A[k] = k == 0 ? (double)Lk[0] : (double)Lk[k] + C.dck[k];
    float s, e[K], Lmax;
    if constexpr (K == 2) {
      const bool one = A[1] > A[0];
      const float es = exp_arg(-fabs(A[1] - A[0]));
      e[0] = one ? es : 1.0f;
      e[1] = one ? 1.0f : es;
      if constexpr (M::HAS_TLIN) {
        e[0] *= Gk[0];
        e[1] *= Gk[1];
        s = e[0] + e[1];
      } else {
        s = 1.0f + es;
      }
      Lmax = one ? Lk[1] : Lk[0];
      acc.t[CB] += one ? 1.0f : 0.0f;
    } else {
      int ks = 0;
      double Mx = A[0];
#pragma unroll
      for (int k = 1; k < K; ++k) {
        ks = A[k] > Mx ? k : ks;
        Mx = fmax(Mx, A[k]);
      }
      s = 0.0f;
      Lmax = Lk[0];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        e[k] = exp_arg(A[k] - Mx);
        if constexpr (M::HAS_TLIN) e[k] *= Gk[k];
        s += e[k];
        Lmax = ks == k ? Lk[k] : Lmax;
        if (k > 0) acc.t[CB + k - 1] += ks == k ? 1.0f : 0.0f;
      }
    }
    // the log-likelihood part without constants: the largest term's L'
    acc.t[0] += rootsum + Lmax;
    if constexpr (M::HAS_LIN) {
      acc.P *= s * gprod;
      acc.bad += !(gprod > 0.0f);
    } else {
      acc.P *= s;
    }
    if constexpr (GRAD) {
      const float inv = rcp_f32(s);
      float r[K];
#pragma unroll
      for (int k = 0; k < K; ++k) r[k] = e[k] * inv;
#pragma unroll
      for (int k = 0; k < K - 1; ++k) acc.t[M::TERM_BASE + k] += r[k];  // the last: N minus the others
      static_for<L>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        using Sl = typename M::template S<l>;
        constexpr int off = M::template leaf_off<l>();
        if constexpr (Sl::root) {
#pragma unroll
          for (int p = 0; p < Sl::Leaf::NP; ++p) acc.t[M::LEAF_BASE + off + p] += phi[off + p];
        } else {
          float R = 0.0f;
          if constexpr (M::FLAT) {
            R = r[M::template term_of<l>()];
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) R += ((C.mask[k] >> l) & 1) ? r[k] : 0.0f;
          }
#pragma unroll
          for (int p = 0; p < Sl::Leaf::NP; ++p)
            acc.t[M::LEAF_BASE + off + p] = fmaf(R, phi[off + p], acc.t[M::LEAF_BASE + off + p]);
        }
      });
    }
  }
}

// event-pass types of a compiled model
// BHHH accumulator (FP64 pass): the gradient sums of Acc plus the second
// moments sum_i v_i v_i^T (upper triangle, row by row) of each event's
// score features v = (r_0 .. r_{K-1} if K > 1, then R_l phi_lp).  The score
// of an event is affine in v with per-point coefficients, s_i = c0 + A v_i,
// so sum_i s_i s_i^T follows from these moments after the reduction.  Each
// event is evaluated into a fresh Acc and folded in.
template <class M>
struct AccBhhh {
  static constexpr int NA = M::template NA<true>;
  static constexpr int NT = M::K > 1 ? M::K : 0;  // responsibilities in v
  static constexpr int NVF = NT + M::NPT;
  static constexpr int NM = NVF * (NVF + 1) / 2;
  Acc<M, true> run;
  double mom[NM];
  __device__ void init() {
    run.init();
#pragma unroll
    for (int j = 0; j < NM; ++j) mom[j] = 0.0;
  }
  __device__ void begin_tile() { run.begin_tile(); }
  __device__ void end_tile() { run.end_tile(); }
  __device__ void finalize(double (&v)[NA + NM]) {
    run.finalize(reinterpret_cast<double(&)[NA]>(v));
#pragma unroll
    for (int j = 0; j < NM; ++j) v[NA + j] = mom[j];
  }
};

template <class M, bool GRAD>
__device__ inline void model_event(const double (&x)[M::NOBS], const Consts<M>& C, AccBhhh<M>& acc) {
  static_assert(GRAD, "the BHHH pass is a gradient pass");
  using AB = AccBhhh<M>;
  Acc<M, true> ev;
  ev.init();
  model_event<M, true>(x, C, ev);
#pragma unroll
  for (int j = 0; j < AB::NA; ++j) acc.run.a[j] += ev.a[j];
  if constexpr (M::NEED_PROD) acc.run.P *= ev.P;
  acc.run.bad += ev.bad;
  double v[AB::NVF];
  if constexpr (AB::NT > 0) {
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < M::K - 1; ++k) {
      v[k] = ev.a[M::TERM_BASE + k];
      rs += v[k];
    }
    v[M::K - 1] = 1.0 - rs;  // the responsibilities of an event sum to 1
  }
#pragma unroll
  for (int j = 0; j < M::NPT; ++j) v[AB::NT + j] = ev.a[M::LEAF_BASE + j];
  int m = 0;
#pragma unroll
  for (int i = 0; i < AB::NVF; ++i)
#pragma unroll
    for (int j = i; j < AB::NVF; ++j, ++m) acc.mom[m] = fma(v[i], v[j], acc.mom[m]);
}

// Weighted events: each event is evaluated into a fresh accumulator of the
// unweighted shape, whose log-domain sum and running product give its
// log-density (one logarithm per event: a weighted sum cannot be folded
// into a product of mantissas), and is added with its weight.
template <class M, bool GRAD>
struct AccW {
  using B = typename M::Base;
  static constexpr int NA = B::template NA<GRAD>;
  double a[NA];
  int bad;
  __device__ void init() {
#pragma unroll
    for (int j = 0; j < NA; ++j) a[j] = 0.0;
    bad = 0;
  }
  __device__ void begin_tile() {}
  __device__ void end_tile() {}
  __device__ void finalize(double (&v)[NA]) {
#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = a[j];
  }
};

template <class M, bool GRAD>
__device__ inline void model_event(const double (&x)[M::NOBS], const Consts<typename M::Base>& C,
                                   AccW<M, GRAD>& acc) {
  using B = typename M::Base;
  constexpr int NA = AccW<M, GRAD>::NA;
  Acc<B, GRAD> e;
  e.init();
  model_event<B, GRAD>(reinterpret_cast<const double(&)[B::NOBS]>(x), C, e);
  const double w = x[B::NOBS];
  double lp = e.a[0];
  // one event's product is s times the root linear factors: a normal
  // double when the density is valid.  Otherwise the logarithm's own values
  // (-inf at 0, +inf at +inf, NaN below 0 or at NaN) are selected as
  // constants: a select between two logarithms would evaluate both.
  if constexpr (B::NEED_PROD) {
    const double P = e.P;
    const bool fin = P > 0.0 && P <= 1.7976931348623157e308;
    const double lt = log_pos_tab(fin ? P : 1.0, g_log_tab);
    const double inv = P == 0.0 ? -__builtin_inf() : (P > 0.0 ? __builtin_inf() : __builtin_nan(""));
    lp += fin ? lt : inv;
  }
  acc.a[0] = fma(w, lp, acc.a[0]);
#pragma unroll
  for (int j = 1; j < NA; ++j) acc.a[j] = fma(w, e.a[j], acc.a[j]);
  acc.bad += e.bad;
}

template <class M, bool GRAD>
struct Pass {
  using C = std::conditional_t<M::PREC == 1, Consts32<M>, Consts<M>>;
  using A = std::conditional_t<M::PREC == 1, Acc32<M, GRAD>, Acc<M, GRAD>>;
};
template <class B, bool GRAD>
struct Pass<Weighted<B>, GRAD> {
  using C = Consts<B>;
  using A = AccW<Weighted<B>, GRAD>;
};

}  // namespace nllmi
